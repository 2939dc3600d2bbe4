"""GPU parity of the learned warm start network (BF16 MFMA, FP32 accumulation)
against the FP64 oracle evaluated with the same BF16-rounded weights.

Tolerance: the GPU rounds every GEMM input activation to BF16 (8 bits of
mantissa, relative spacing 2^-8 = 3.9e-3); through three layers the outputs
and gradients carry a few such roundings, so blocks are compared in relative
norm at 3e-2 and in direction (cosine >= 0.999)."""
import numpy as np
import pytest
import torch

from oracle import mpnn as N
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


def _sample(n=3000, seed=2):
    c = sphere_cluster(n, seed)
    og = O.collide(c["pos"], c["radius"])
    oa = O.assemble(og)
    ot = O.build_tree(og)
    v, _ = O.pcg(oa, c["force"], "tree", O.tree_factor(og, ot))
    vprev = v + 0.3 * np.random.default_rng(seed).normal(size=v.shape) * v.std()
    return c, og, vprev, v


def _oracle(theta, c, og, vprev, v, scales):
    ee = N.entry_edges(og.rowptr, og.col, og.ei, og.ej)
    rows, e = N.edge_features(og.rowptr, og.col, og.ei, og.ej, og.w, og.u, ee, scales[2])
    return N.loss_grad(theta, c["force"], vprev, v, og.rowptr, og.col, e, rows, scales)


def test_forward_and_gradients_match_oracle(ctx):
    c, og, vprev, v = _sample()
    scales = (float(c["force"].std()), float(v.std()), 0.1)
    theta = N.init_params(4) + 0.02 * np.random.default_rng(1).normal(size=N.param_count())
    theta_b = N.bf16_round(theta)
    M = P.Mpnn(ctx)
    M.set_params(theta, *scales)
    g = ctx.collide(to_dev(c["pos"]), to_dev(c["radius"]))
    F, Vp, V = to_dev(c["force"]), to_dev(vprev), to_dev(v)
    vh = host(M.forward(g, F, Vp))
    L, grad, out = _oracle(theta_b, c, og, vprev, v, scales)
    vo = out * scales[1]
    assert np.linalg.norm(vh - vo) <= 3e-2 * np.linalg.norm(vo)
    lg, gg = M.grad(g, F, Vp, V)
    gg = host(gg).astype(np.float64)
    assert abs(lg - L) <= 3e-2 * L
    pg, po = N.unpack(gg), N.unpack(grad)
    for name, _ in N.LAYOUT:
        a, b = pg[name].ravel(), po[name].ravel()
        nb = np.linalg.norm(b)
        assert np.linalg.norm(a - b) <= 3e-2 * nb + 1e-12, name
        if nb > 0:
            assert a @ b / (np.linalg.norm(a) * nb) >= 0.999, name


def test_gradient_is_deterministic(ctx):
    c, og, vprev, v = _sample(2000, 3)
    M = P.Mpnn(ctx)
    M.set_params(N.init_params(2), 1.0, float(v.std()), 0.1)
    g = ctx.collide(to_dev(c["pos"]), to_dev(c["radius"]))
    args = (g, to_dev(c["force"]), to_dev(vprev), to_dev(v))
    l1, g1 = M.grad(*args)
    l2, g2 = M.grad(*args)
    assert l1 == l2 and torch.equal(g1, g2)


def test_training_lowers_the_loss(ctx):
    c, og, vprev, v = _sample(4000, 5)
    M = P.Mpnn(ctx)
    M.set_params(N.init_params(0), float(c["force"].std()), float(v.std()), 0.1)
    g = ctx.collide(to_dev(c["pos"]), to_dev(c["radius"]))
    args = (g, to_dev(c["force"]), to_dev(vprev), to_dev(v))
    losses = [M.train_step(*args, 1e-3) for _ in range(60)]
    assert losses[-1] < 0.5 * losses[0], losses[::10]


def test_adam_updates_match_oracle(ctx):
    """Each training update (sgp_mpnn_train_step) against the oracle's Adam
    step applied to the same gradient (sgp_mpnn_grad at the same parameters:
    bitwise the gradient the update uses) from the same parameters, with the
    moments carried in FP64 from the GPU's gradients.  Tolerance: the
    update runs in FP32, whose 1 - beta2^t for t = 2, 3 loses ~3e-5 to
    cancellation, so 1e-4 of the step size lr (Adam's steps are about lr)
    plus one FP32 rounding of the parameter; a wrong moment, bias
    correction, eps placement or sign moves a step by a large fraction."""
    c, og, vprev, v = _sample(3000, 7)
    M = P.Mpnn(ctx)
    M.set_params(N.init_params(3), float(c["force"].std()), float(v.std()), 0.1)
    g = ctx.collide(to_dev(c["pos"]), to_dev(c["radius"]))
    args = (g, to_dev(c["force"]), to_dev(vprev), to_dev(v))
    lr = 1e-3
    th = host(M.get_params()).astype(np.float64)
    m1 = m2 = np.zeros_like(th)
    for t in range(1, 4):
        _, gr = M.grad(*args)
        gr = host(gr).astype(np.float64)
        M.train_step(*args, lr)
        th_gpu = host(M.get_params()).astype(np.float64)
        ref, m1, m2 = N.adam_step(th, gr, m1, m2, t, lr)
        err = np.abs(th_gpu - ref)
        tol = 1e-4 * lr + 2.0 ** -23 * np.abs(ref)
        print(f"adam step {t}: max |gpu - oracle| {err.max():.3e}, moved {np.abs(th_gpu - th).max():.3e}", flush=True)
        assert np.all(err <= tol), (t, int(np.argmax(err - tol)))
        assert np.count_nonzero(th_gpu != th) >= 0.5 * np.count_nonzero(gr) > 0
        th = th_gpu


def test_energy_gradients_match_oracle(ctx):
    """Energy loss ||v_hat - v||^2_Gamma / ||v||^2_Gamma: value and gradient
    against the oracle (Gamma from the oracle's assembly), same tolerance."""
    c, og, vprev, v = _sample(3000, 6)
    oa = O.assemble(og)
    scales = (float(c["force"].std()), float(v.std()), 0.1)
    theta = N.init_params(8) + 0.02 * np.random.default_rng(3).normal(size=N.param_count())
    theta_b = N.bf16_round(theta)
    M = P.Mpnn(ctx)
    M.set_params(theta, *scales)
    g = ctx.collide(to_dev(c["pos"]), to_dev(c["radius"]))
    A = ctx.assemble_gamma(g)
    lg, gg = M.grad(g, to_dev(c["force"]), to_dev(vprev), to_dev(v), A)
    L, grad, _ = _oracle_energy(theta_b, c, og, oa, vprev, v, scales)
    assert abs(lg - L) <= 3e-2 * abs(L), (lg, L)
    pg, po = N.unpack(host(gg).astype(np.float64)), N.unpack(grad)
    for name, _ in N.LAYOUT:
        a, b = pg[name].ravel(), po[name].ravel()
        nb = np.linalg.norm(b)
        assert np.linalg.norm(a - b) <= 3e-2 * nb + 1e-12, name
        if nb > 0:
            assert a @ b / (np.linalg.norm(a) * nb) >= 0.999, name


def _oracle_energy(theta, c, og, oa, vprev, v, scales):
    ee = N.entry_edges(og.rowptr, og.col, og.ei, og.ej)
    rows, e = N.edge_features(og.rowptr, og.col, og.ei, og.ej, og.w, og.u, ee, scales[2])
    return N.loss_grad(theta, c["force"], vprev, v, og.rowptr, og.col, e, rows, scales, lambda x: O.spmv(oa, x))


def test_warm_start_picks_the_lowest_energy(ctx):
    """x0 is, of v_prev, the network's guess and zero, the first one of lowest
    energy 0.5 x'Gx - x'F (energies checked against the oracle's product);
    all three branches exercised."""
    c, og, vprev, v = _sample(2000, 7)
    oa = O.assemble(og)
    F = c["force"]

    def energy(x):
        a, b = 0.5 * np.sum(x * O.spmv(oa, x)), np.sum(x * F)
        return a - b, abs(a) + abs(b)

    g = ctx.collide(to_dev(c["pos"]), to_dev(c["radius"]))
    A = ctx.assemble_gamma(g)
    garbage = 50.0 * np.random.default_rng(9).normal(size=v.shape)
    # a zero network guesses 0 (energy 0): it beats a garbage v_prev and loses
    # to the solution itself (the lowest energy); a network with inflated
    # weights guesses far off, and with a garbage v_prev the zero start wins
    cases = [(N.init_params(1), vprev, None), (np.zeros(N.param_count()), garbage, 1),
             (N.init_params(1), v, 0), (50.0 * N.init_params(3), garbage, 2)]
    for theta, vp, expect in cases:
        M = P.Mpnn(ctx)
        M.set_params(theta, float(F.std()), float(v.std()), 0.1)
        vh = host(M.forward(g, to_dev(F), to_dev(vp)))
        x0, info = M.warm_start(g, A, to_dev(F), to_dev(vp))
        en, sn = energy(vh)
        ep, sp = energy(vp)
        assert abs(info["energy_net"] - en) <= 1e-10 * sn
        assert abs(info["energy_prev"] - ep) <= 1e-10 * sp
        pick = 0 if (info["energy_prev"] <= info["energy_net"] and info["energy_prev"] <= 0.0) else \
            (1 if info["energy_net"] <= 0.0 else 2)
        assert info["used_net"] == (pick == 1) and info["used_zero"] == (pick == 2)
        if expect is not None:
            assert pick == expect, (pick, expect, en, ep)
        want = (vp, vh, np.zeros_like(vp))[pick]
        assert np.array_equal(host(x0), want)


def test_hand_computed_three_cell_forward(ctx):
    """The hand-worked three-cell case of the oracle's pins (neighbour term
    h_j, edge direction n_ij = (r_i - r_j)/d_ij, overlap feature), through the
    GPU network: every input and weight is exact in BF16, so only the overlap
    feature (w/sW = 1 + 2^-49 rounds to 1) differs from the exact answer."""
    from tests.test_oracle_mpnn import hand_case
    pos, R, F, vprev, scales, theta, want = hand_case()
    M = P.Mpnn(ctx)
    M.set_params(theta, *scales)
    g = ctx.collide(to_dev(pos), to_dev(R))
    vh = host(M.forward(g, to_dev(F), to_dev(vprev)))
    assert np.allclose(vh, want, rtol=1e-6, atol=1e-6), vh
