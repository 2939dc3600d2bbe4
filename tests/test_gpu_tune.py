"""Launch-shape knobs and the autotuner, through the C ABI.

check_every, tail_max and hipGraph replay must leave results bitwise
unchanged (they change when and how kernels are issued, never what they
compute); spmv_waves changes only the summation order of p.q, so results
agree to CG's rounding spread.  Graph replays are checked against eager
solves several times, with other eager work and synchronisations between
them."""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from workloads import sphere_cluster, batched_instance

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


def _system(ctx, n=20000, seed=11):
    c = sphere_cluster(n, seed)
    g = ctx.collide(to_dev(c["pos"]), to_dev(c["radius"]))
    A = ctx.assemble_gamma(g)
    T = ctx.build_tree(g)
    return c, g, A, T


def test_defaults_and_rejections(ctx):
    assert ctx.tune_get("check_every") == 2 and ctx.tune_get("tail_max") == 2200
    assert ctx.tune_get("graph") == 0 and ctx.tune_get("spmv_waves") == 4
    assert ctx.tune_get("light_height") == 0 and ctx.tune_get("light_cap") == 512
    assert ctx.tune_get("spmv_form") == 1 and ctx.tune_get("tail_side") == 1 and ctx.tune_get("prefetch") == 1
    for key, bad in (("check_every", 0), ("tail_max", -1), ("graph", 2), ("spmv_waves", 3), ("nope", 1),
                     ("light_height", -1), ("light_cap", 0), ("spmv_form", 2), ("tail_side", 2),
                     ("prefetch", -1)):
        with pytest.raises(P.SgpError):
            ctx.tune(key, bad)


def test_graph_replay_is_bitwise_eager(ctx):
    c, g, A, T = _system(ctx)
    M = ctx.factor_tree(g, T)
    F = to_dev(c["force"])
    ctx.tune("check_every", 4)
    v0, i0 = ctx.pcg_solve(A, M, F)
    ctx.tune("graph", 1)
    for rep in range(3):
        v1, i1 = ctx.pcg_solve(A, M, F)
        assert i1["iters"] == i0["iters"] and torch.equal(v0, v1), rep
        # eager work and a synchronisation between replays
        ctx.tune("graph", 0)
        v2, _ = ctx.pcg_solve(A, M, F, fixed_iters=5)
        torch.cuda.synchronize()
        ctx.tune("graph", 1)
    # FP32-inner refinement runs its inner CG through the same path
    ctx.tune("graph", 0)
    w0, j0 = ctx.pcg_solve(A, M, F, precision="f32ir", inner_rtol=1e-4)
    ctx.tune("graph", 1)
    w1, j1 = ctx.pcg_solve(A, M, F, precision="f32ir", inner_rtol=1e-4)
    assert j0["iters"] == j1["iters"] and torch.equal(w0, w1)
    og = O.collide(c["pos"], c["radius"])
    check_velocity(host(v1), i1["iters"], O.assemble(og), c["force"], O.tree_factor(og, O.build_tree(og)))


def test_graph_replay_batched(ctx):
    sizes = [3000, 500, 12000, 40]
    parts = [batched_instance(k + 1, n_override=s) for k, s in enumerate(sizes)]
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    pos = to_dev(np.concatenate([p["pos"] for p in parts]))
    R = to_dev(np.concatenate([p["radius"] for p in parts]))
    F = to_dev(np.concatenate([p["force"] for p in parts]))
    g = ctx.collide_batched(off, pos, R)
    A = ctx.assemble_gamma(g)
    M = ctx.factor_tree(g, ctx.build_tree(g))
    ctx.tune("check_every", 4)
    v0, i0 = ctx.pcg_solve_batched(A, M, off, F)
    ctx.tune("graph", 1)
    for _ in range(2):
        v1, i1 = ctx.pcg_solve_batched(A, M, off, F)
        assert [a["iters"] for a in i0] == [b["iters"] for b in i1]
        assert torch.equal(v0, v1)


def test_check_every_and_tail_max_are_bitwise_neutral(ctx):
    c, g, A, T = _system(ctx, 30000, 12)
    F = to_dev(c["force"])
    M = ctx.factor_tree(g, T)
    ref, iref = ctx.pcg_solve(A, M, F)
    for ce in (1, 3, 32):
        ctx.tune("check_every", ce)
        v, i = ctx.pcg_solve(A, M, F)
        assert i["iters"] == iref["iters"] and torch.equal(v, ref), ce
    ctx.tune("check_every", 2)
    for tm in (0, 300):
        ctx.tune("tail_max", tm)
        M2 = ctx.factor_tree(g, T)
        v, i = ctx.pcg_solve(A, M2, F)
        assert i["iters"] == iref["iters"] and torch.equal(v, ref), tm
        b = torch.randn_like(F)
        assert torch.equal(ctx.prec_apply(M2, b), ctx.prec_apply(M, b)), tm


def test_spmv_waves_change_rounding_only(ctx):
    c, g, A, T = _system(ctx, 30000, 13)
    F = to_dev(c["force"])
    M = ctx.factor_tree(g, T)
    x = torch.randn_like(F)
    q4 = ctx.spmv(A, x)
    ref, iref = ctx.pcg_solve(A, M, F)
    for wv in (2, 8):
        ctx.tune("spmv_waves", wv)
        assert torch.equal(ctx.spmv(A, x), q4), wv    # the product itself is unchanged
        v, i = ctx.pcg_solve(A, M, F)
        assert abs(i["iters"] - iref["iters"]) <= 1
        if i["iters"] == iref["iters"]:
            assert float(torch.linalg.vector_norm(v - ref) / torch.linalg.vector_norm(ref)) <= 1e-8


def test_autotuner_choice_solves(ctx):
    from paper_2410_04512_amd import autotune
    c, g, A, T = _system(ctx, 20000, 14)
    F = to_dev(c["force"])
    res = autotune.tune(ctx, g, T, A, F, fixed_iters=10, repeats=1)
    assert res["schedule"] in autotune.SCHEDULES and res["tail_max"] in autotune.TAIL_MAX
    assert ctx.tune_get("spmv_waves") == res["spmv_waves"] and ctx.tune_get("graph") == res["graph"]
    assert ctx.tune_get("check_every") == res["check_every"]
    v, info = ctx.pcg_solve(A, res["prec"], F)
    assert info["status"] == 0 and info["relres_true"] <= 1.0001e-8
    print({k: v_ for k, v_ in res.items() if k not in ("prec",)})


@pytest.mark.parametrize("lh,cap", [(0, 512), (4, 1), (32, 64), (32, 512), (1000, 512)])
def test_light_subtree_sweeps_match_oracle(ctx, lh, cap):
    """The rake-only start with its one-workgroup-per-subtree sweeps (and the
    extremes: off, one vertex per workgroup, a tree raked away completely):
    the tree solve against the oracle's, FP64 and FP32, and a converged CG."""
    c, g, A, T = _system(ctx, 6000, 15)
    ctx.tune("light_height", lh)
    ctx.tune("light_cap", cap)
    M = ctx.factor_tree(g, T)
    og = O.collide(c["pos"], c["radius"])
    fo = O.tree_factor(og, O.build_tree(og))
    b = np.random.default_rng(lh).normal(size=(6000, 3))
    zo = O.tree_solve(fo, b)
    z = host(ctx.prec_apply(M, to_dev(b)))
    assert np.linalg.norm(z - zo) <= 1e-10 * np.linalg.norm(zo)
    F = to_dev(c["force"])
    v, info = ctx.pcg_solve(A, M, F)
    assert info["status"] == 0 and info["relres_true"] <= 1.0001e-8
    check_velocity(host(v), info["iters"], O.assemble(og), c["force"], fo)
    w, i32 = ctx.pcg_solve(A, M, F, precision="f32ir", inner_rtol=1e-4)
    assert i32["status"] == 0 and i32["relres_true"] <= 1.0001e-8


@pytest.mark.parametrize("cap,tail", [(1, 2200), (64, 2200), (512, 2200), (512, 256), (512, 0), (4096, 2200)])
def test_mid_step_sweeps_match_oracle(ctx, cap, tail):
    """The mid elimination steps swept one workgroup per group of components
    (60k cells: steps from the third on, up to the default tail), with one
    component per workgroup, small and default packing, groups too large for
    the LDS sweeps (4,096-vertex packing: the generic workgroup sweeps run),
    and with the tail smaller than the default (steps between the mid range
    and the tail as launches of their own) or off: the tree solve against the
    oracle's, FP64 and FP32, a converged CG, and results that do not depend on
    the tail."""
    c, g, A, T = _system(ctx, 60000, 21)
    ctx.tune("light_cap", cap)
    ctx.tune("tail_max", tail)
    try:
        M = ctx.factor_tree(g, T)
        og = O.collide(c["pos"], c["radius"])
        fo = O.tree_factor(og, O.build_tree(og))
        b = np.random.default_rng(cap).normal(size=(60000, 3))
        zo = O.tree_solve(fo, b)
        z = host(ctx.prec_apply(M, to_dev(b)))
        assert np.linalg.norm(z - zo) <= 1e-10 * np.linalg.norm(zo)
        F = to_dev(c["force"])
        v, info = ctx.pcg_solve(A, M, F)
        assert info["status"] == 0 and info["relres_true"] <= 1.0001e-8
        check_velocity(host(v), info["iters"], O.assemble(og), c["force"], fo)
        w, i32 = ctx.pcg_solve(A, M, F, precision="f32ir", inner_rtol=1e-4)
        assert i32["status"] == 0 and i32["relres_true"] <= 1.0001e-8
        if tail != 2200:   # the grouping is fixed by the schedule: the tail changes nothing
            ctx.tune("tail_max", 2200)
            M2 = ctx.factor_tree(g, T)
            v2, info2 = ctx.pcg_solve(A, M2, F)
            assert info2["iters"] == info["iters"] and torch.equal(v, v2)
    finally:
        ctx.tune("light_cap", 512)
        ctx.tune("tail_max", 2200)


def test_light_subtrees_batched(ctx):
    """A batch of separate trees (several of them raked away completely)."""
    sizes = [3000, 20, 9000, 1, 700]
    parts = [batched_instance(k + 3, n_override=s) for k, s in enumerate(sizes)]
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    pos = to_dev(np.concatenate([p["pos"] for p in parts]))
    R = to_dev(np.concatenate([p["radius"] for p in parts]))
    F = np.concatenate([p["force"] for p in parts])
    g = ctx.collide_batched(off, pos, R)
    A = ctx.assemble_gamma(g)
    M = ctx.factor_tree(g, ctx.build_tree(g))
    v, infos = ctx.pcg_solve_batched(A, M, off, to_dev(F))
    vh = host(v)
    for k, p in enumerate(parts):
        og = O.collide(p["pos"], p["radius"])
        assert infos[k]["status"] == 0
        check_velocity(vh[off[k]:off[k + 1]], infos[k]["iters"], O.assemble(og), p["force"],
                       O.tree_factor(og, O.build_tree(og)))


@pytest.mark.parametrize("n,seed", [(6000, 16), (30000, 17)])
def test_edge_form_product_and_solve(ctx, n, seed):
    """The product from the contacts' (w, u) against the stored blocks and the
    oracle's assembled Gamma (FP64 rounding only), and CG with either form."""
    c, g, A, T = _system(ctx, n, seed)
    og = O.collide(c["pos"], c["radius"])
    oa = O.assemble(og)
    x = np.random.default_rng(seed).normal(size=(n, 3))
    ref = O.spmv(oa, x)
    ctx.tune("spmv_form", 0)
    q0 = host(ctx.spmv(A, to_dev(x)))
    ctx.tune("spmv_form", 1)
    q1 = host(ctx.spmv(A, to_dev(x)))
    for q in (q0, q1):
        assert np.linalg.norm(q - ref) <= 1e-14 * np.linalg.norm(ref)
    M = ctx.factor_tree(g, T)
    fo = O.tree_factor(og, O.build_tree(og))
    F = to_dev(c["force"])
    for form in (0, 1):
        ctx.tune("spmv_form", form)
        v, info = ctx.pcg_solve(A, M, F)
        assert info["status"] == 0 and info["relres_true"] <= 1.0001e-8
        check_velocity(host(v), info["iters"], oa, c["force"], fo)
        w, i32 = ctx.pcg_solve(A, M, F, precision="f32ir", inner_rtol=1e-4)
        assert i32["status"] == 0 and i32["relres_true"] <= 1.0001e-8


def test_edge_form_with_isolated_cells(ctx):
    """Rows without contacts (isolated cells, a batch of singletons) are owned
    by the product's last wave: q_i = g_med p_i for them."""
    sizes = [1, 1, 500, 1, 64, 1, 1]
    parts = [batched_instance(k + 9, n_override=s) for k, s in enumerate(sizes)]
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    pos = np.concatenate([p["pos"] + 100.0 * k for k, p in enumerate(parts)])
    R = np.concatenate([p["radius"] for p in parts])
    g = ctx.collide_batched(off, to_dev(pos), to_dev(R))
    A = ctx.assemble_gamma(g)
    x = np.random.default_rng(3).normal(size=(pos.shape[0], 3))
    ctx.tune("spmv_form", 0)
    q0 = host(ctx.spmv(A, to_dev(x)))
    ctx.tune("spmv_form", 1)
    q1 = host(ctx.spmv(A, to_dev(x)))
    assert np.linalg.norm(q1 - q0) <= 1e-14 * np.linalg.norm(q0)
    for k, s in enumerate(sizes):
        if s == 1:
            i = off[k]
            assert np.allclose(q1[i], 1e-3 * x[i], rtol=1e-15, atol=0)


@pytest.mark.parametrize("n,seed", [(20000, 21), (60000, 22)])
def test_fused_first_step_is_bitwise_neutral(ctx, n, seed):
    """The first elimination step inside the CG's vector passes (knob
    fuse_step0, on by default) gives the same bits as its own launches: FP64
    from zero and from a warm start, and the FP32-inner refinement."""
    c, g, A, T = _system(ctx, n, seed)
    F = to_dev(c["force"])
    M = ctx.factor_tree(g, T)
    info = M.info()
    # the first step runs as launches of its own here (below the tail, no light steps)
    assert info["tail_step"] > 0 and info["light_steps"] == 0
    assert ctx.tune_get("fuse_step0") == 1
    x0 = torch.randn_like(F) * 1e-3
    runs = {}
    for fuse in (1, 0):
        ctx.tune("fuse_step0", fuse)
        runs[fuse] = (ctx.pcg_solve(A, M, F), ctx.pcg_solve(A, M, F, x0.clone(), use_x0=True),
                      ctx.pcg_solve(A, M, F, precision="f32ir"))
    for (va, ia), (vb, ib) in zip(runs[1], runs[0]):
        assert ia["iters"] == ib["iters"] and ia.get("outer_iters") == ib.get("outer_iters")
        assert torch.equal(va, vb)
    ctx.tune("fuse_step0", 1)
    with pytest.raises(P.SgpError):
        ctx.tune("fuse_step0", 2)


def test_fused_first_step_batched(ctx):
    sizes = [3000, 500, 12000, 40, 25000, 1]
    parts = [batched_instance(k + 1, n_override=s) for k, s in enumerate(sizes)]
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    pos = to_dev(np.concatenate([p["pos"] for p in parts]))
    R = to_dev(np.concatenate([p["radius"] for p in parts]))
    F = to_dev(np.concatenate([p["force"] for p in parts]))
    g = ctx.collide_batched(off, pos, R)
    A = ctx.assemble_gamma(g)
    M = ctx.factor_tree(g, ctx.build_tree(g))
    assert M.info()["tail_step"] > 0
    v1, i1 = ctx.pcg_solve_batched(A, M, off, F)
    ctx.tune("fuse_step0", 0)
    v0, i0 = ctx.pcg_solve_batched(A, M, off, F)
    ctx.tune("fuse_step0", 1)
    assert [a["iters"] for a in i1] == [b["iters"] for b in i0]
    assert all(a["status"] == 0 for a in i1)
    assert torch.equal(v0, v1)


@pytest.mark.parametrize("n,seed", [(60000, 41), (200000, 42)])
def test_mid_steps_in_lds_are_bitwise_neutral(ctx, n, seed):
    """The mid steps swept with their slots and x in LDS (knob mid_lds, on by
    default) give the same bits as the generic workgroup sweeps: the apply,
    the FP64 solve and the FP32 refinement."""
    c, g, A, T = _system(ctx, n, seed)
    F = to_dev(c["force"])
    M = ctx.factor_tree(g, T)
    info = M.info()
    assert info["tail_step"] >= 6 and info["light_steps"] == 0   # mid steps exist below the tail
    b = torch.randn_like(F)
    runs = {}
    for on in (1, 0):
        ctx.tune("mid_lds", on)
        runs[on] = (ctx.prec_apply(M, b), ctx.pcg_solve(A, M, F), ctx.pcg_solve(A, M, F, precision="f32ir"))
    ctx.tune("mid_lds", 1)
    assert torch.equal(runs[1][0], runs[0][0])
    for (va, ia), (vb, ib) in zip(runs[1][1:], runs[0][1:]):
        assert ia["iters"] == ib["iters"] and torch.equal(va, vb)
    if n <= 60000:   # and the apply against the oracle's tree solve
        og = O.collide(c["pos"], c["radius"])
        z = O.tree_solve(O.tree_factor(og, O.build_tree(og)), host(b))
        assert np.linalg.norm(host(runs[1][0]) - z) <= 1e-10 * np.linalg.norm(z)


def test_mid_steps_in_lds_batched(ctx):
    sizes = [40000, 3000, 70000, 500]
    parts = [batched_instance(k + 11, n_override=s) for k, s in enumerate(sizes)]
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    pos = to_dev(np.concatenate([p["pos"] for p in parts]))
    R = to_dev(np.concatenate([p["radius"] for p in parts]))
    F = to_dev(np.concatenate([p["force"] for p in parts]))
    g = ctx.collide_batched(off, pos, R)
    A = ctx.assemble_gamma(g)
    M = ctx.factor_tree(g, ctx.build_tree(g))
    v1, i1 = ctx.pcg_solve_batched(A, M, off, F)
    ctx.tune("mid_lds", 0)
    v0, i0 = ctx.pcg_solve_batched(A, M, off, F)
    ctx.tune("mid_lds", 1)
    assert [a["iters"] for a in i1] == [b["iters"] for b in i0]
    assert all(a["status"] == 0 for a in i1)
    assert torch.equal(v0, v1)


@pytest.mark.parametrize("n,seed", [(60000, 43), (1500, 44)])
def test_tail_side_update_is_bitwise_neutral(ctx, n, seed):
    """x += alpha p run by extra workgroups of the tail launch (knob
    tail_side, on by default) gives the same bits as the CG's own update
    pass: FP64 solves to a tolerance, at fixed counts, from a warm start, on
    the error bound, with chunk graphs, and the FP32 refinement."""
    c, g, A, T = _system(ctx, n, seed)
    F = to_dev(c["force"])
    M = ctx.factor_tree(g, T)
    assert M.info()["tail_step"] < M.steps()   # the sweeps have a tail
    x0 = torch.randn_like(F)
    ctx.tune("small_solve", 0)
    runs = {}
    for on in (1, 0):
        ctx.tune("tail_side", on)
        r = [ctx.pcg_solve(A, M, F), ctx.pcg_solve(A, M, F, fixed_iters=7),
             ctx.pcg_solve(A, M, F, v=x0.clone(), use_x0=True), ctx.pcg_solve(A, M, F, rtol=1e-6, stop="error"),
             ctx.pcg_solve(A, M, F, precision="f32ir")]
        ctx.tune("graph", 1)
        r.append(ctx.pcg_solve(A, M, F, check_every=3))
        ctx.tune("graph", 0)
        runs[on] = r
    ctx.tune("tail_side", 1)
    ctx.tune("small_solve", 1)
    for (va, ia), (vb, ib) in zip(runs[1], runs[0]):
        assert ia["iters"] == ib["iters"] and ia["status"] == ib["status"] == 0
        assert torch.equal(va, vb)
    if n <= 2000:
        og = O.collide(c["pos"], c["radius"])
        check_velocity(host(runs[1][0][0]), runs[1][0][1]["iters"], O.assemble(og), c["force"],
                       O.tree_factor(og, O.build_tree(og)))


def test_tail_side_update_batched(ctx):
    """Instances converge at different iterations: the side update stops
    with each, as the CG's own pass does."""
    sizes = [40000, 3000, 70000, 500, 9000]
    parts = [batched_instance(k + 21, n_override=s) for k, s in enumerate(sizes)]
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    pos = to_dev(np.concatenate([p["pos"] for p in parts]))
    R = to_dev(np.concatenate([p["radius"] for p in parts]))
    F = to_dev(np.concatenate([p["force"] for p in parts]))
    g = ctx.collide_batched(off, pos, R)
    A = ctx.assemble_gamma(g)
    M = ctx.factor_tree(g, ctx.build_tree(g))
    v1, i1 = ctx.pcg_solve_batched(A, M, off, F)
    ctx.tune("tail_side", 0)
    v0, i0 = ctx.pcg_solve_batched(A, M, off, F)
    ctx.tune("tail_side", 1)
    assert [a["iters"] for a in i1] == [b["iters"] for b in i0]
    assert len({a["iters"] for a in i1}) > 1 and all(a["status"] == 0 for a in i1)
    assert torch.equal(v0, v1)


def test_tail_prefetch_is_bitwise_neutral(ctx):
    """The tail's constants prefetched into L2 by the launch before it (knob
    prefetch, on by default): the apply, the FP64 solve and the FP32
    refinement give the same bits with it off."""
    c, g, A, T = _system(ctx, 60000, 45)
    F = to_dev(c["force"])
    M = ctx.factor_tree(g, T)
    assert M.info()["tail_step"] < M.steps()
    b = torch.randn_like(F)
    runs = {}
    for on in (1, 0):
        ctx.tune("prefetch", on)
        runs[on] = (ctx.prec_apply(M, b), ctx.pcg_solve(A, M, F), ctx.pcg_solve(A, M, F, precision="f32ir"))
    ctx.tune("prefetch", 1)
    assert torch.equal(runs[1][0], runs[0][0])
    for (va, ia), (vb, ib) in zip(runs[1][1:], runs[0][1:]):
        assert ia["iters"] == ib["iters"] and torch.equal(va, vb)


def test_blocks_assembled_on_first_use(ctx):
    """Gamma's 3x3 blocks are assembled only for the block-CSR product: a
    matrix assembled under the edge form and then multiplied in block form
    gives that form's product (within rounding of the edge form's, and bit
    for bit the product of a matrix assembled under the block form); block
    Jacobi, built from the diagonal blocks of the edge form, is unchanged;
    a graph collided again before the blocks are built is refused."""
    c = sphere_cluster(20000, 46)
    pos, R = to_dev(c["pos"]), to_dev(c["radius"])
    g = ctx.collide(pos, R)
    A = ctx.assemble_gamma(g)
    x = torch.randn_like(pos)
    y1 = ctx.spmv(A, x)
    ctx.tune("spmv_form", 0)
    try:
        y0 = ctx.spmv(A, x)   # blocks built now
        A0 = ctx.assemble_gamma(g)   # blocks built with the assembly
        assert torch.equal(ctx.spmv(A0, x), y0)
        assert float((y0 - y1).abs().max() / y1.abs().max()) <= 1e-13
        F = to_dev(c["force"])
        M = ctx.factor_tree(g, ctx.build_tree(g))
        v0, i0 = ctx.pcg_solve(A, M, F)
        assert i0["status"] == 0
    finally:
        ctx.tune("spmv_form", 1)
    J = ctx.make_jacobi(A)
    v, info = ctx.pcg_solve(A, J, to_dev(c["force"]))
    assert info["status"] == 0
    # a second graph handle keeps the first one's version intact; collide the
    # same handle again with moved cells, then ask for the blocks
    A2 = ctx.assemble_gamma(g)
    ctx.collide(pos + 0.01, R, 32, g)
    ctx.tune("spmv_form", 0)
    try:
        with pytest.raises(P.SgpError):
            ctx.spmv(A2, x)
    finally:
        ctx.tune("spmv_form", 1)
