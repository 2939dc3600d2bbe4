"""Pins of the oracle's learned warm start network (FP64): manual backward
against central finite differences, permutation equivariance, a closed-form
special case."""
import numpy as np
import pytest

from oracle import mpnn as N
from oracle import oracle as O
from workloads import sphere_cluster


def _setup(n=40, seed=1):
    c = sphere_cluster(n, seed)
    g = O.collide(c["pos"], c["radius"])
    ee = N.entry_edges(g.rowptr, g.col, g.ei, g.ej)
    rows, e = N.edge_features(g.rowptr, g.col, g.ei, g.ej, g.w, g.u, ee, 0.1)
    rng = np.random.default_rng(seed)
    F = c["force"]
    vprev = rng.normal(size=(n, 3))
    v = rng.normal(size=(n, 3))
    return g, rows, e, F, vprev, v


def test_entry_edges_match_oracle_assembly_order():
    c = sphere_cluster(300, 2)
    g = O.collide(c["pos"], c["radius"])
    ee = N.entry_edges(g.rowptr, g.col, g.ei, g.ej)
    rows = np.repeat(np.arange(g.n), np.diff(g.rowptr))
    assert np.array_equal(np.minimum(rows, g.col), g.ei[ee])
    assert np.array_equal(np.maximum(rows, g.col), g.ej[ee])


def test_gradients_match_central_differences():
    g, rows, e, F, vprev, v = _setup()
    theta = N.init_params(3)
    # biases nonzero so every parameter matters
    theta = theta + 0.05 * np.random.default_rng(0).normal(size=theta.shape)
    scales = (1.0, 2.0, 0.1)
    L, grad, _ = N.loss_grad(theta, F, vprev, v, g.rowptr, g.col, e, rows, scales)
    rng = np.random.default_rng(1)
    idx = rng.choice(theta.size, size=400, replace=False)
    h = 1e-6
    num = np.empty(idx.size)
    for k, i in enumerate(idx):
        tp = theta.copy(); tp[i] += h
        tm = theta.copy(); tm[i] -= h
        Lp = N.loss_grad(tp, F, vprev, v, g.rowptr, g.col, e, rows, scales)[0]
        Lm = N.loss_grad(tm, F, vprev, v, g.rowptr, g.col, e, rows, scales)[0]
        num[k] = (Lp - Lm) / (2 * h)
    err = np.abs(num - grad[idx])
    assert np.all(err <= 1e-6 * np.abs(grad[idx]).max() + 1e-7 * np.abs(num)), err.max()
    # every parameter block received a nonzero gradient somewhere
    p = N.unpack(grad)
    for name, _ in N.LAYOUT:
        assert np.abs(p[name]).max() > 0, name


def test_permutation_equivariance():
    c = sphere_cluster(60, 4)
    perm = np.random.default_rng(0).permutation(60)
    theta = N.init_params(1)
    rng = np.random.default_rng(5)
    vprev = rng.normal(size=(60, 3))
    outs = []
    for P_ in (np.arange(60), perm):
        g = O.collide(c["pos"][P_], c["radius"][P_])
        ee = N.entry_edges(g.rowptr, g.col, g.ei, g.ej)
        rows, e = N.edge_features(g.rowptr, g.col, g.ei, g.ej, g.w, g.u, ee, 0.1)
        out, _ = N.forward(theta, c["force"][P_], vprev[P_], g.rowptr, g.col, e, rows, (1.0, 1.0, 0.1))
        outs.append(out)
    inv = np.empty(60, int); inv[perm] = np.arange(60)
    assert np.allclose(outs[1][inv], outs[0], rtol=1e-12, atol=1e-12)


def test_isolated_cell_closed_form():
    """A cell with no contacts sees no messages: out = h3 W_out + b_out with h
    built from its own features only (computed here with the layers written out)."""
    pos = np.array([[0.0, 0, 0], [10.0, 0, 0]])
    g = O.collide(pos, np.ones(2))
    assert g.m == 0
    theta = N.init_params(7)
    p = N.unpack(theta)
    F = np.array([[1.0, -2.0, 0.5], [0.0, 0.0, 0.0]])
    vprev = np.array([[0.3, 0.1, -0.2], [0.0, 0.0, 0.0]])
    rows, e = N.edge_features(g.rowptr, g.col, g.ei, g.ej, g.w, g.u, np.zeros(0, int), 1.0)
    out, _ = N.forward(theta, F, vprev, g.rowptr, g.col, e.reshape(0, 4), rows, (1.0, 1.0, 1.0))
    h = np.maximum(np.concatenate([F[0], vprev[0]]) @ p["W_in"] + p["b_in"], 0)
    for l in range(3):
        U = np.concatenate([h, np.zeros(64)]) @ p[f"W_u{l}"] + p[f"b_u{l}"]
        h = h + np.maximum(U, 0)
    assert np.allclose(out[0], h @ p["W_out"] + p["b_out"], rtol=1e-14)


def test_bf16_rounding():
    # bf16 keeps 7 fraction bits: the spacing just above 1 is 2^-7
    a = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 2 ** -7 + 3 * 2 ** -9, -3.14159, 0.0, 1e-30, 1.0 + 2 ** -7 + 2 ** -9])
    r = N.bf16_round(a)
    assert r[0] == 1.0 and r[1] == 1.0          # half a spacing: tie to even
    assert r[2] == 1.0 + 2 ** -6                # 3/4 of a spacing: up
    assert r[6] == 1.0 + 2 ** -7                # 1/4 of a spacing: down
    assert abs(r[3] + 3.140625) < 1e-12
    assert r[4] == 0.0


def _gamma(g):
    A = O.assemble(g).dense()
    return A, (lambda x: (A @ x.reshape(-1)).reshape(-1, 3))


def test_energy_loss_is_the_gamma_norm_error():
    """With v the exact solution (dense solve), the energy loss equals
    ||v_hat - v||^2_Gamma / ||v||^2_Gamma computed from the dense matrix, is 0
    at v_hat = v and 1 at v_hat = 0."""
    g, rows, e, F, vprev, _ = _setup(60, 3)
    A, mv = _gamma(g)
    v = np.linalg.solve(A, F.reshape(-1)).reshape(-1, 3)
    sV = 0.7
    out = np.random.default_rng(2).normal(size=v.shape)
    L, _ = N.energy_loss_and_dout(out, v, F, mv, sV)
    d = (sV * out - v).reshape(-1)
    ref = d @ A @ d / (v.reshape(-1) @ A @ v.reshape(-1))
    assert abs(L - ref) <= 1e-10 * ref
    assert abs(N.energy_loss_and_dout(v / sV, v, F, mv, sV)[0]) <= 1e-10
    assert abs(N.energy_loss_and_dout(np.zeros_like(v), v, F, mv, sV)[0] - 1.0) <= 1e-12


def test_energy_gradients_match_central_differences():
    g, rows, e, F, vprev, _ = _setup()
    A, mv = _gamma(g)
    v = np.linalg.solve(A, F.reshape(-1)).reshape(-1, 3)
    theta = N.init_params(5) + 0.05 * np.random.default_rng(3).normal(size=N.param_count())
    scales = (1.0, float(v.std()), 0.1)
    L, grad, _ = N.loss_grad(theta, F, vprev, v, g.rowptr, g.col, e, rows, scales, mv)
    rng = np.random.default_rng(4)
    idx = rng.choice(theta.size, size=300, replace=False)
    h = 1e-6
    num = np.empty(idx.size)
    for k, i in enumerate(idx):
        tp = theta.copy(); tp[i] += h
        tm = theta.copy(); tm[i] -= h
        Lp = N.loss_grad(tp, F, vprev, v, g.rowptr, g.col, e, rows, scales, mv)[0]
        Lm = N.loss_grad(tm, F, vprev, v, g.rowptr, g.col, e, rows, scales, mv)[0]
        num[k] = (Lp - Lm) / (2 * h)
    err = np.abs(num - grad[idx])
    assert np.all(err <= 1e-6 * np.abs(grad[idx]).max() + 1e-7 * np.abs(num)), err.max()


def hand_case():
    """A three-cell chain 0 - 1 - 2 along x (centres 1.9 apart, unit radii:
    neighbours overlap by w = 2 - 1.9, cells 0 and 2 do not touch) and
    parameters that route single features through one message-passing layer,
    so that the output is known by hand:
      h_i[0]  = relu(F_i,x / sF)                          (W_in)
      z_p[1]  = h_j[0],  z_p[3] = n_ij,x,  z_p[5] = w_ij / sW   (W_b, W_c of layer 0)
      h_i[2], h_i[4], h_i[6] += the sums over i's neighbours of those (W_u)
      out_i   = (h_i[2], h_i[4], h_i[6]),  v_hat = sV out    (W_out)
    Layers 1 and 2 are zero and leave h unchanged.  With F_x = (1, 2, 4),
    n_ij = (r_i - r_j)/d_ij and the chain's geometry:
      out[:, 0] = sum of the neighbours' F_x      = (2, 1 + 4, 2)
      out[:, 1] = sum of max(n_ij,x, 0)           = (0, 1, 1)
      out[:, 2] = sum of w_ij / sW                = (w, 2 w, w) / sW
    (the cell's own feature in place of its neighbour's would give
    (1, 4, 4) in column 0; n pointing i -> j would give (1, 1, 0) in column 1)."""
    pos = np.array([[0.0, 0.0, 0.0], [1.9, 0.0, 0.0], [3.8, 0.0, 0.0]])
    R = np.ones(3)
    F = np.array([[1.0, 0.5, -0.25], [2.0, -1.0, 0.75], [4.0, 0.0, 1.5]])
    vprev = np.array([[0.1, 0.2, 0.3], [-0.4, 0.5, -0.6], [0.7, -0.8, 0.9]])
    sF, sV, sW = 1.0, 2.0, 0.1
    p = {name: np.zeros(shape) for name, shape in N.LAYOUT}
    H = N.HID
    p["W_in"][0, 0] = 1.0
    p["W_b0"][0, 1] = 1.0
    p["W_c0"][1, 3] = 1.0
    p["W_c0"][0, 5] = 1.0
    p["W_u0"][H + 1, 2] = 1.0
    p["W_u0"][H + 3, 4] = 1.0
    p["W_u0"][H + 5, 6] = 1.0
    p["W_out"][2, 0] = 1.0
    p["W_out"][4, 1] = 1.0
    p["W_out"][6, 2] = 1.0
    w = 2.0 - 1.9
    want = sV * np.array([[2.0, 0.0, w / sW], [5.0, 1.0, 2 * w / sW], [2.0, 1.0, w / sW]])
    return pos, R, F, vprev, (sF, sV, sW), N.pack(p), want


def test_hand_computed_three_cell_forward():
    pos, R, F, vprev, scales, theta, want = hand_case()
    g = O.collide(pos, R)
    assert g.m == 2 and list(g.ei) == [0, 1] and list(g.ej) == [1, 2]
    ee = N.entry_edges(g.rowptr, g.col, g.ei, g.ej)
    rows, e = N.edge_features(g.rowptr, g.col, g.ei, g.ej, g.w, g.u, ee, scales[2])
    out, _ = N.forward(theta, F, vprev, g.rowptr, g.col, e, rows, scales)
    assert np.allclose(scales[1] * out, want, rtol=1e-12, atol=1e-15), scales[1] * out


def test_adam_step_closed_forms():
    """The optimiser's update against values worked out by hand from its
    definition: the first step from zero moments moves every parameter by
    lr g / (|g| + eps) (the bias corrections give back g and g^2); a constant
    gradient keeps that step at every t; two different gradients give the
    rational moments below; eps sits outside the root; no gradient, no move."""
    lr, eps = 1e-3, 1e-8
    th0 = np.array([0.5, -1.0, 2.0, 0.0, 3.0])
    g = np.array([0.25, -4.0, 1e-9, 0.0, 7.0])
    z = np.zeros_like(g)
    th1, m1, m2 = N.adam_step(th0, g, z, z, 1, lr)
    assert np.allclose(th1 - th0, -lr * g / (np.abs(g) + eps), rtol=1e-12, atol=0.0)
    # |g| = 1e-9: a step of lr / 11 (eps under the root would give ~lr 1e-5)
    assert abs((th1[2] - th0[2]) + lr / 11.0) <= 1e-12 * lr
    assert th1[3] == th0[3]
    # fifty steps of one constant gradient
    th, a, b = th0, z, z
    for t in range(1, 51):
        th, a, b = N.adam_step(th, g, a, b, t, lr)
    assert np.allclose(th - th0, -50 * lr * g / (np.abs(g) + eps), rtol=1e-10, atol=1e-15)
    # g = 1 then g = -2: corrected moments -11/19 and 4999/1999 at t = 2
    s, a, b = N.adam_step(np.array([0.0]), np.array([1.0]), np.zeros(1), np.zeros(1), 1, lr)
    assert abs(s[0] + lr / (1.0 + eps)) <= 1e-15
    s2, a, b = N.adam_step(s, np.array([-2.0]), a, b, 2, lr)
    step2 = -lr * (-11.0 / 19.0) / (np.sqrt(4999.0 / 1999.0) + eps)
    assert abs((s2[0] - s[0]) - step2) <= 1e-12 * abs(step2)
