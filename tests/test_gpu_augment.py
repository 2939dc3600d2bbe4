"""GPU parity of the augmented maximum spanning tree (Section 3.1) and its
nested solve (flexible CG around an inner tree-PCG; Sections 3 and 5)
against the oracle: pieces and added contacts bit for bit; with a nearly
exact inner solve the outer iterations and velocity of plain PCG with P'; with
the paper's inner tolerance 0.1 the tolerance met and the solution within
the forward-error bound."""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from workloads import sphere_cluster

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_2410_04512_amd")
from tests.gpu_util import host, to_dev  # noqa: E402


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = P.Context()
    yield c
    c.close()


def _both(ctx, n, seed, parts, inner):
    c = sphere_cluster(n, seed)
    pos, R, F = to_dev(c["pos"]), to_dev(c["radius"]), to_dev(c["force"])
    g = ctx.collide(pos, R)
    T = ctx.build_tree(g)
    M = ctx.factor_augmented(g, T, parts=parts, inner_rtol=inner)
    A = ctx.assemble_gamma(g)
    og = O.collide(c["pos"], c["radius"])
    ot = O.build_tree(og)
    aug, piece, added = O.augment(og, ot, parts if parts > 0 else None)
    return c, g, T, M, A, F, og, ot, aug, piece, added


@pytest.mark.parametrize("n,seed,parts", [(3000, 1, 0), (3000, 2, 3), (3000, 3, 40), (20000, 4, 0)])
def test_pieces_and_added_contacts_bit_exact(ctx, n, seed, parts):
    c, g, T, M, A, F, og, ot, aug, piece, added = _both(ctx, n, seed, parts, 0.1)
    npc, nad, gp, ga = ctx.prec_augmented(M, n)
    print(f"augment: n={n} parts={parts}: {npc} pieces, {nad} added contacts", flush=True)
    assert np.array_equal(host(gp), piece)
    assert np.array_equal(host(ga), added)
    assert npc == np.unique(piece).size


def test_nearly_exact_inner_solve_matches_the_oracle(ctx):
    c, g, T, M, A, F, og, ot, aug, piece, added = _both(ctx, 3000, 5, 6, 1e-12)
    assert added.size > 0
    v, info = ctx.pcg_solve(A, M, F)
    oa = O.assemble(og)
    xo, io = O.fcg(oa, O.assemble_edges(og, aug), O.tree_factor(og, ot), c["force"], inner_tol=1e-12)
    print(f"augment exact inner: outer {info['iters']} (oracle {io.iters}), inner {info['inner_iters']} "
          f"(oracle {io.outer})", flush=True)
    assert info["status"] == 0 and abs(info["iters"] - io.iters) <= 1
    err = np.linalg.norm(host(v) - xo) / np.linalg.norm(xo)
    assert err <= 1e-8 if info["iters"] == io.iters else err <= 2e3 * 1e-8, err


@pytest.mark.parametrize("n,seed", [(3000, 6), (20000, 7)])
def test_paper_inner_tolerance(ctx, n, seed):
    c, g, T, M, A, F, og, ot, aug, piece, added = _both(ctx, n, seed, 0, 0.1)
    v, info = ctx.pcg_solve(A, M, F)
    oa = O.assemble(og)
    xo, io = O.fcg(oa, O.assemble_edges(og, aug), O.tree_factor(og, ot), c["force"], inner_tol=0.1)
    print(f"augment n={n}: outer {info['iters']} (oracle {io.iters}), inner {info['inner_iters']} "
          f"(oracle {io.outer})", flush=True)
    assert info["status"] == 0 and info["relres_true"] <= 1.0001e-8
    assert abs(info["iters"] - io.iters) <= 3
    r = c["force"] - O.spmv(oa, host(v))
    assert np.linalg.norm(r) <= 1.0001e-8 * np.linalg.norm(c["force"])
    assert np.linalg.norm(host(v) - xo) <= 2e3 * 1e-8 * np.linalg.norm(xo)


def test_refused_forms(ctx):
    c = sphere_cluster(500, 8)
    pos, R, F = to_dev(c["pos"]), to_dev(c["radius"]), to_dev(c["force"])
    g = ctx.collide(pos, R)
    M = ctx.factor_augmented(g, ctx.build_tree(g))
    A = ctx.assemble_gamma(g)
    for kw in ({"precision": "f32ir"}, {"fixed_iters": 5}):
        with pytest.raises(P.SgpError):
            ctx.pcg_solve(A, M, F, **kw)
    with pytest.raises(P.SgpError):
        ctx.pcg_solve_batched(A, M, [0, 200, 500], F)
    with pytest.raises(P.SgpError):
        ctx.factor_augmented(g, ctx.build_forest(g, pos, R, 64))
