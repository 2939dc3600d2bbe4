"""Learned warm start over overdamped time steps (orchestration only).

Each step of the cell model (Section 2: forces from the current contacts,
the friction solve, an explicit Euler position update) runs through libsgp:
collide -> forces -> assemble_gamma -> build_tree -> factor_tree -> pcg_solve
-> euler.  The warm start is not part of the paper's method: a message-passing
network maps (F, v_prev) on the collision graph to a guess x0 for the solve.
CG to the same relative residual still decides the result, so the network
only changes how many iterations the solve needs.  The network is trained on the energy
norm of its error, ||v_hat - v||_Gamma, the norm CG's progress is measured in;
at run time the start of lowest energy 0.5 x' Gamma x - x' F among v_prev
(the fallback), the network's guess and zero is used.

Protocol: steps 1..n_train solve from x0 = v_prev and keep (graph, Gamma, F,
v_prev, v) as training samples; the network is then trained on the GPU (Adam
over shuffled samples); steps n_train+1..n_steps solve three times from the
same state (from zero, from v_prev, from the learned warm start) and advance
with the learned run's velocity.  Every solve and every network pass runs in
libsgp; the only host arithmetic here is the bookkeeping of the report.
"""
from __future__ import annotations

import time

import numpy as np
import torch

from .sgp import Context, Mpnn


def _now(ctx):
    torch.cuda.synchronize(ctx.dev())
    return time.perf_counter()


def step_system(ctx: Context, pos, radius, noise, k_rep, schedule="contract"):
    """Graph, forces, Gamma and the tree preconditioner at the current positions."""
    g = ctx.collide(pos, radius)
    F = ctx.forces(g, noise, k_rep)
    A = ctx.assemble_gamma(g)
    M = ctx.factor_tree(g, ctx.build_tree(g), schedule=schedule)
    return g, F, A, M


def train(model: Mpnn, samples, epochs, lr, seed=0, log=None):
    """Adam on the energy loss over samples (g, A, F, v_prev, v) in a seeded
    shuffled order each epoch; returns the mean loss of every epoch."""
    rng = np.random.default_rng(seed)
    hist = []
    for ep in range(epochs):
        losses = []
        for k in rng.permutation(len(samples)):
            g, A, F, vp, v = samples[k]
            losses.append(model.train_step(g, F, vp, v, lr, A))
        hist.append(float(np.mean(losses)))
        if log:
            log(f"train epoch {ep + 1}/{epochs}: mean loss {hist[-1]:.4e}")
    return hist


def run(ctx: Context, pos, radius, noise_fn, n_steps=200, n_train=100, dt=0.01, k_rep=5.0,
        epochs=20, lr=1e-3, rtol=1e-8, seed=0, schedule="contract", log=None, on_test_step=None):
    """Run the protocol.  `pos` (device [n][3] FP64) is advanced in place;
    `noise_fn(step, n)` returns the active force of a step (host or device).
    `on_test_step(t, pos, F, x0, v, iters)`, if given, sees every test
    step's positions (before the update), forces, learned initial guess,
    solved velocity and the solve's iteration count.  Returns per-step
    records and the training history."""
    n = pos.shape[0]
    dev = pos.device
    v_prev = torch.zeros((n, 3), dtype=torch.float64, device=dev)
    samples, train_rec, test_rec = [], [], []

    def noise(t):
        return torch.as_tensor(noise_fn(t, n), dtype=torch.float64).to(dev).contiguous()

    for t in range(1, n_train + 1):
        g, F, A, M = step_system(ctx, pos, radius, noise(t), k_rep, schedule)
        t0 = _now(ctx)
        v, info = ctx.pcg_solve(A, M, F, v=v_prev.clone(), use_x0=True, rtol=rtol)
        ms = (_now(ctx) - t0) * 1e3
        train_rec.append({"step": t, "iters": info["iters"], "ms": ms, "relres_true": info["relres_true"]})
        samples.append((g, A, F, v_prev, v))
        ctx.euler(pos, v, dt)
        v_prev = v
        if log and (t % 10 == 0 or t == 1):
            log(f"step {t}: {info['iters']} iterations from v_prev, {ms:.1f} ms")

    F_all = torch.stack([s[2] for s in samples])
    V_all = torch.stack([s[4] for s in samples])
    scales = (float(F_all.std()), float(V_all.std()), 0.1)
    del F_all, V_all
    model = Mpnn(ctx)
    model.set_params(_init_params(seed, model.param_count()), *scales)
    t0 = _now(ctx)
    hist = train(model, samples, epochs, lr, seed, log)
    train_s = _now(ctx) - t0
    samples.clear()

    for t in range(n_train + 1, n_steps + 1):
        g, F, A, M = step_system(ctx, pos, radius, noise(t), k_rep, schedule)
        # the plain method from zero, and from the previous step's velocity
        t0 = _now(ctx)
        v_z, iz = ctx.pcg_solve(A, M, F, rtol=rtol)
        ms_z = (_now(ctx) - t0) * 1e3
        t0 = _now(ctx)
        v_a, ia = ctx.pcg_solve(A, M, F, v=v_prev.clone(), use_x0=True, rtol=rtol)
        ms_a = (_now(ctx) - t0) * 1e3
        # learned warm start (network pass + energy pick) and its solve
        t0 = _now(ctx)
        x0, ws = model.warm_start(g, A, F, v_prev)
        x0_kept = x0.clone() if on_test_step else None
        v_b, ib = ctx.pcg_solve(A, M, F, v=x0, use_x0=True, rtol=rtol)
        ms_b = (_now(ctx) - t0) * 1e3
        if on_test_step:
            on_test_step(t, pos, F, x0_kept, v_b, ib["iters"])
        # report only: the energy of the solution, E* = -0.5 v' F, scales the
        # energies of the guesses to relative Gamma-norm errors (zero start = 1)
        e_star = -0.5 * float(torch.dot(v_b.reshape(-1), F.reshape(-1)))
        test_rec.append({"step": t, "iters_zero": iz["iters"], "iters_prev": ia["iters"], "iters_learned": ib["iters"],
                         "ms_zero": ms_z, "ms_prev": ms_a, "ms_learned": ms_b, "used_net": ws["used_net"],
                         "used_zero": ws["used_zero"],
                         "err_net": (ws["energy_net"] - e_star) / -e_star,
                         "err_prev": (ws["energy_prev"] - e_star) / -e_star,
                         "relres_true": max(iz["relres_true"], ia["relres_true"], ib["relres_true"]),
                         "status": max(abs(iz["status"]), abs(ia["status"]), abs(ib["status"]))})
        ctx.euler(pos, v_b, dt)
        v_prev = v_b
        if log and (t % 10 == 0 or t == n_train + 1):
            r = test_rec[-1]
            log(f"step {t}: iterations {iz['iters']} from zero, {ia['iters']} from v_prev, {ib['iters']} learned; "
                f"energy error net {r['err_net']:.3f} v_prev {r['err_prev']:.3f}; "
                f"{ms_z:.1f} / {ms_a:.1f} / {ms_b:.1f} ms")
    return {"train": train_rec, "test": test_rec, "loss_history": hist, "train_seconds": train_s,
            "scales": scales, "model": model}


def summary(res):
    """Means over the test steps and the learned warm start's iteration and
    wall-time ratios against the v_prev warm start and the zero start."""
    te = res["test"]

    def mean(k):
        return float(np.mean([r[k] for r in te]))

    out = {"test_steps": len(te)}
    for k in ("iters_zero", "iters_prev", "iters_learned", "ms_zero", "ms_prev", "ms_learned", "err_net", "err_prev"):
        out["mean_" + k] = mean(k)
    out["iter_ratio_vs_prev"] = out["mean_iters_learned"] / out["mean_iters_prev"]
    out["wall_ratio_vs_prev"] = out["mean_ms_learned"] / out["mean_ms_prev"]
    out["iter_ratio_vs_zero"] = out["mean_iters_learned"] / out["mean_iters_zero"]
    out["wall_ratio_vs_zero"] = out["mean_ms_learned"] / out["mean_ms_zero"]
    out["net_used"] = int(sum(r["used_net"] for r in te))
    out["zero_used"] = int(sum(r["used_zero"] for r in te))
    out["max_relres_true"] = float(max(r["relres_true"] for r in te))
    out["all_converged"] = all(r["status"] == 0 for r in te)
    out["train_seconds"] = res["train_seconds"]
    out["final_loss"] = res["loss_history"][-1] if res["loss_history"] else None
    return out


def _init_params(seed, count):
    """Glorot-uniform weights and zero biases in the layer layout of the network
    (width 64, three layers; the same layout the C ABI documents), with the
    output layer zero: the untrained network guesses 0, the zero start, and
    training moves it from there."""
    hid, nin, ne, nout = 64, 6, 4, 3
    shapes = [("W", nin, hid), ("b", hid)]
    for _ in range(3):
        shapes += [("W", hid, hid), ("W", hid, hid), ("W", ne, hid), ("b", hid), ("W", 2 * hid, hid), ("b", hid)]
    shapes += [("Z", hid, nout), ("b", nout)]
    rng = np.random.default_rng(seed)
    parts = []
    for s in shapes:
        if s[0] == "b":
            parts.append(np.zeros(s[1]))
        elif s[0] == "Z":
            parts.append(np.zeros(s[1] * s[2]))
        else:
            lim = np.sqrt(6.0 / (s[1] + s[2]))
            parts.append(rng.uniform(-lim, lim, s[1] * s[2]))
    theta = np.concatenate(parts)
    assert theta.size == count
    return theta
