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
