"""Helpers shared by the GPU tests: run the library's chain on seeded inputs."""
import numpy as np
import torch

import paper_2410_04512_amd as P


def to_dev(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)


def host(t):
    return t.detach().cpu().numpy()


def gpu_chain(ctx, c, schedule="contract", prec="tree", max_deg=32, **solve):
    pos, R, F = to_dev(c["pos"]), to_dev(c["radius"]), to_dev(c["force"])
    g = ctx.collide(pos, R, max_deg)
    A = ctx.assemble_gamma(g)
    T = M = None
    if prec == "tree":
        T = ctx.build_tree(g)
        M = ctx.factor_tree(g, T, schedule=schedule)
    elif prec == "jacobi":
        M = ctx.make_jacobi(A)
    v, info = ctx.pcg_solve(A, M, F, **solve)
    return {"g": g, "A": A, "T": T, "M": M, "v": v, "info": info, "F": F, "pos": pos, "R": R}


def check_velocity(v_gpu, iters_gpu, A, F, factor, x0=None, rtol=1e-8, prec="tree"):
    """Velocity parity under the same x0, stopping rule and preconditioner.

    Equal iteration counts: compare with the oracle's solution.  Counts one
    apart (the residual crossed the tolerance within rounding of it): compare
    with the oracle run for exactly the GPU's iteration count.  Returns the
    relative error."""
    from oracle import oracle as O
    xo, io = O.pcg(A, F, prec, factor, x0=x0)
    if io.iters != iters_gpu:
        assert abs(io.iters - iters_gpu) <= 1, (io.iters, iters_gpu)
        xo, io = O.pcg(A, F, prec, factor, x0=x0, fixed_iters=iters_gpu)
    den = max(np.linalg.norm(xo), 1e-300)
    err = np.linalg.norm(v_gpu - xo) / den
    assert err <= rtol, err
    return err
