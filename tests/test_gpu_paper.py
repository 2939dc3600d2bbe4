"""GPU parity on the paper's own benchmark geometries (Section 5.1): cells of
radius 0.5 with the Hertz contact area, friction coefficients g_par = 2e6,
g_perp = 8e7 and g_med = 3e4 or 3e3, the known-solution force
F = Gamma x_true.  Graph (with the Hertz w), Gamma and tree bit-exact; the
velocities of CG without a preconditioner, with block Jacobi and with the
tree against the oracle on the same inputs: within 1e-8, or, where hundreds
of iterations on these stiff systems amplify rounding beyond that, within 10x
the spread between the oracle and a second CPU implementation of the same
recurrence (gpu_util.check_velocity_spread)."""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from workloads import paper as W

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_2410_04512_amd")
from tests.gpu_util import check_velocity_spread, host, to_dev  # noqa: E402


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = P.Context()
    c.set_contact_model("hertz")
    yield c
    c.close()


@pytest.mark.parametrize("kind,n", [("hex", 3000), ("hex_ill", 3000), ("random", 3000), ("dumbbell", 3000),
                                    ("hex", 20000)])
def test_paper_geometry_parity(ctx, kind, n):
    c = W.paper_cells(kind, n, 2)
    gp, gq, gm = c["g_par"], c["g_perp"], c["g_med"]
    print(f"paper: {kind} n={n}", flush=True)
    g = ctx.collide(to_dev(c["pos"]), to_dev(c["radius"]))
    og = O.collide(c["pos"], c["radius"], area="hertz")
    e = {k: host(v) for k, v in ctx.graph_export(g).items()}
    for f in ("rowptr", "col", "ei", "ej", "w", "u"):
        assert np.array_equal(e[f], getattr(og, f)), f
    A = ctx.assemble_gamma(g, gp, gq, gm)
    oa = O.assemble(og, gp, gq, gm)
    b = {k: host(v) for k, v in ctx.bsr_export(A).items()}
    assert np.array_equal(b["val"], oa.val) and np.array_equal(b["bcol"], oa.bcol)
    T = ctx.build_tree(g)
    ot = O.build_tree(og)
    t = {k: host(v) for k, v in ctx.tree_export(T, n).items()}
    assert np.array_equal(t["tree_edge"], ot.tree_edge) and np.array_equal(t["parent"], ot.parent)
    fo = O.tree_factor(og, ot, gp, gq, gm)
    F = O.spmv(oa, c["x_true"])
    precs = {"none": None, "jacobi": ctx.make_jacobi(A), "tree": ctx.factor_tree(g, T, gp, gq, gm)}
    for name, M in precs.items():
        v, info = ctx.pcg_solve(A, M, to_dev(F))
        assert info["status"] == 0, (name, info)
        err, spread = check_velocity_spread(host(v), info["iters"], oa, F, fo if name == "tree" else None,
                                            prec=name)
        tail = f" (second CPU implementation's spread {spread:.2e})" if spread is not None else ""
        print(f"paper: {kind} n={n} {name}: {info['iters']} iterations, velocity error vs the oracle {err:.2e}"
              + tail, flush=True)
