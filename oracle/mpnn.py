"""FP64 reference of the learned warm start: a message-passing network over
the collision graph mapping (F, v_prev) to a velocity guess.

TEST INFRASTRUCTURE ONLY (oracle): the GPU library never imports this.

The method in the paper ends at the PCG solve; the warm start is an addition.
The network (hidden width 64, three message-passing layers):

  x_i   = [F_i / sF, v_prev,i / sV]                          (6 features)
  e_p   = [w_ij / sW, n_ij]  for the CSR entry p = (i, j),  n_ij = (r_i - r_j)/d_ij
  h     = relu(x W_in + b_in)
  layer l = 1..3:
     z_p  = h_i W_a + b_m + h_j W_b + e_p W_c        (the message MLP on [h_i, h_j, e_p])
     m_p  = relu(z_p)
     a_i  = sum over the entries of row i of m_p      (ascending neighbour)
     U    = [h, a] W_u + b_u
     h    = h + relu(U)
  out   = h W_out + b_out;   v_hat = sV * out
  loss  = mean over i and components of (out_i - v_i / sV)^2        (MSE), or
  loss  = ||v_hat - v||^2_Gamma / ||v||^2_Gamma                       (energy)

The energy loss is the Gamma-norm error that CG's convergence depends on.
With Gamma v = F it equals (v_hat' Gamma v_hat - 2 v_hat' F + v' F) / (v' F),
written in that form so that its gradient is exactly 2 sV (Gamma v_hat - F) /
(v' F) with respect to `out`: it needs the residual of the guess, not v.

`forward` keeps what the manual `backward` needs; gradients are pinned by
central finite differences in the tests, and `adam_step` (one update of
the optimiser) by values worked out by hand.  The weights after a whole
training run, and so the trained network's guesses, are parity unpinned:
each update is checked, but the BF16 forward changes every gradient slightly
and the differences compound over a run (the CG solve that follows a guess
is checked against the solver oracle instead).
"""
from __future__ import annotations

import numpy as np

HID = 64
LAYERS = 3
NIN = 6
NEDGE = 4
NOUT = 3

# flat parameter layout (FP32 on the GPU, FP64 here): name, shape
LAYOUT = [("W_in", (NIN, HID)), ("b_in", (HID,))]
for _l in range(LAYERS):
    LAYOUT += [(f"W_a{_l}", (HID, HID)), (f"W_b{_l}", (HID, HID)), (f"W_c{_l}", (NEDGE, HID)),
               (f"b_m{_l}", (HID,)), (f"W_u{_l}", (2 * HID, HID)), (f"b_u{_l}", (HID,))]
LAYOUT += [("W_out", (HID, NOUT)), ("b_out", (NOUT,))]


def param_count():
    return int(sum(np.prod(s) for _, s in LAYOUT))


def unpack(theta):
    out, k = {}, 0
    for name, shape in LAYOUT:
        size = int(np.prod(shape))
        out[name] = np.asarray(theta[k:k + size], dtype=np.float64).reshape(shape)
        k += size
    return out


def pack(p):
    return np.concatenate([np.asarray(p[name], dtype=np.float64).ravel() for name, _ in LAYOUT])


def init_params(seed=0):
    """Glorot-uniform weights, zero biases (seeded)."""
    rng = np.random.default_rng(seed)
    p = {}
    for name, shape in LAYOUT:
        if name.startswith("b"):
            p[name] = np.zeros(shape)
        else:
            lim = np.sqrt(6.0 / (shape[0] + shape[1]))
            p[name] = rng.uniform(-lim, lim, shape)
    return pack(p)


def edge_features(rowptr, col, ei, ej, w, u, ent_edge, sW):
    """e_p = [w/sW, n] for every CSR entry p = (i, j); n = (r_i - r_j)/d = -u for i < j."""
    n = rowptr.shape[0] - 1
    rows = np.repeat(np.arange(n), np.diff(rowptr))
    sign = np.where(rows < col, -1.0, 1.0)
    e = np.empty((col.shape[0], NEDGE))
    e[:, 0] = w[ent_edge] / sW
    e[:, 1:] = sign[:, None] * u[ent_edge]
    return rows, e


def entry_edges(rowptr, col, ei, ej):
    """Edge id of every CSR entry (the edge list is lexicographic in (i, j), i < j)."""
    n = rowptr.shape[0] - 1
    rows = np.repeat(np.arange(n), np.diff(rowptr))
    a = np.minimum(rows, col)
    b = np.maximum(rows, col)
    key = a.astype(np.int64) * n + b
    ekey = ei.astype(np.int64) * n + ej
    return np.searchsorted(ekey, key)


def relu(x):
    return np.maximum(x, 0.0)


def forward(theta, F, vprev, rowptr, col, e, rows, scales):
    sF, sV, sW = scales
    p = unpack(theta)
    x = np.concatenate([F / sF, vprev / sV], axis=1)
    pre0 = x @ p["W_in"] + p["b_in"]
    h = relu(pre0)
    cache = {"x": x, "pre0": pre0, "layers": []}
    n = F.shape[0]
    for l in range(LAYERS):
        P = h @ p[f"W_a{l}"] + p[f"b_m{l}"]
        Q = h @ p[f"W_b{l}"]
        z = P[rows] + Q[col] + e @ p[f"W_c{l}"]
        m = relu(z)
        a = np.zeros((n, HID))
        np.add.at(a, rows, m)
        U = np.concatenate([h, a], axis=1) @ p[f"W_u{l}"] + p[f"b_u{l}"]
        cache["layers"].append({"h": h, "z": z, "a": a, "U": U})
        h = h + relu(U)
    out = h @ p["W_out"] + p["b_out"]
    cache["h_last"] = h
    return out, cache


def loss_and_dout(out, v, sV):
    t = v / sV
    d = out - t
    L = float(np.mean(d * d))
    return L, 2.0 * d / d.size


def energy_loss_and_dout(out, v, F, gamma_mv, sV):
    """Energy loss and its gradient with respect to `out`; gamma_mv(x) = Gamma x."""
    vh = sV * out
    q = gamma_mv(vh)
    c = float(np.sum(v * F))
    L = (float(np.sum(vh * q)) - 2.0 * float(np.sum(vh * F)) + c) / c
    return L, 2.0 * sV * (q - F) / c


def backward(theta, dout, cache, rowptr, col, e, rows):
    p = unpack(theta)
    g = {name: np.zeros(shape) for name, shape in LAYOUT}
    h = cache["h_last"]
    g["W_out"] = h.T @ dout
    g["b_out"] = dout.sum(axis=0)
    dh = dout @ p["W_out"].T
    n = h.shape[0]
    for l in reversed(range(LAYERS)):
        c = cache["layers"][l]
        hin, z, a, U = c["h"], c["z"], c["a"], c["U"]
        dU = dh * (U > 0)
        cat = np.concatenate([hin, a], axis=1)
        g[f"W_u{l}"] = cat.T @ dU
        g[f"b_u{l}"] = dU.sum(axis=0)
        dcat = dU @ p[f"W_u{l}"].T
        dhin = dh + dcat[:, :HID]
        da = dcat[:, HID:]
        dz = da[rows] * (z > 0)
        dP = np.zeros((n, HID))
        np.add.at(dP, rows, dz)
        dQ = np.zeros((n, HID))
        np.add.at(dQ, col, dz)
        g[f"W_c{l}"] = e.T @ dz
        g[f"b_m{l}"] = dP.sum(axis=0)
        g[f"W_a{l}"] = hin.T @ dP
        g[f"W_b{l}"] = hin.T @ dQ
        dhin = dhin + dP @ p[f"W_a{l}"].T + dQ @ p[f"W_b{l}"].T
        dh = dhin
    dpre0 = dh * (cache["pre0"] > 0)
    g["W_in"] = cache["x"].T @ dpre0
    g["b_in"] = dpre0.sum(axis=0)
    return pack(g)


def loss_grad(theta, F, vprev, v, rowptr, col, e, rows, scales, gamma_mv=None):
    """Loss, gradient and output; the energy loss when gamma_mv is given, else MSE."""
    out, cache = forward(theta, F, vprev, rowptr, col, e, rows, scales)
    if gamma_mv is None:
        L, dout = loss_and_dout(out, v, scales[1])
    else:
        L, dout = energy_loss_and_dout(out, v, F, gamma_mv, scales[1])
    return L, backward(theta, dout, cache, rowptr, col, e, rows), out


def bf16_round(a):
    """Round-to-nearest-even to bfloat16 (kept in float64)."""
    f = np.asarray(a, dtype=np.float32)
    b = f.view(np.uint32).astype(np.uint64)
    lsb = (b >> 16) & 1
    r = ((b + 0x7FFF + lsb) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def adam_step(theta, g, m1, m2, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba, 2015, Algorithm 1), the optimiser that
    trains the network: the moment estimates are exponential averages of the
    gradient and of its square, each divided by (1 - beta^t) to undo their
    start at zero, and every parameter moves by lr times the corrected first
    moment over (the root of the corrected second moment plus eps).  t counts
    updates from 1.  Returns (theta, m1, m2), new arrays in float64."""
    g = np.asarray(g, dtype=np.float64)
    m1 = b1 * np.asarray(m1, dtype=np.float64) + (1.0 - b1) * g
    m2 = b2 * np.asarray(m2, dtype=np.float64) + (1.0 - b2) * g * g
    mh = m1 / (1.0 - b1 ** t)
    vh = m2 / (1.0 - b2 ** t)
    return np.asarray(theta, dtype=np.float64) - lr * mh / (np.sqrt(vh) + eps), m1, m2
