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


def second_cpu_pcg(A, F, prec, factor, k, x0=None):
    """A second CPU implementation of the oracle's PCG (numpy dot products,
    scipy's sparse product, numpy block-Jacobi solves): the same recurrence
    in another summation order, run for exactly k iterations."""
    import scipy.sparse as sp
    from oracle import oracle as O
    S = sp.bsr_matrix((A.val, A.bcol, A.rowptr), shape=(3 * A.n, 3 * A.n)).tocsr()
    b = np.asarray(F, dtype=np.float64).ravel()
    if prec == "tree":
        def msolve(r):
            return O.tree_solve(factor, r).ravel()
    elif prec == "jacobi":
        diag = np.stack([A.val[A.rowptr[i] + np.searchsorted(A.bcol[A.rowptr[i]:A.rowptr[i + 1]], i)]
                         for i in range(A.n)])
        dinv = np.linalg.inv(diag)

        def msolve(r):
            return np.einsum("nab,nb->na", dinv, r.reshape(-1, 3)).ravel()
    else:
        def msolve(r):
            return r.copy()
    x = np.zeros_like(b) if x0 is None else np.asarray(x0, dtype=np.float64).ravel().copy()
    r = b - S @ x
    z = msolve(r)
    p = z.copy()
    rho = r @ z
    for _ in range(k):
        q = S @ p
        a = rho / (p @ q)
        x += a * p
        r -= a * q
        z = msolve(r)
        rn = r @ z
        p = z + (rn / rho) * p
        rho = rn
    return x.reshape(-1, 3)


def check_velocity_spread(v_gpu, iters_gpu, A, F, factor, prec="tree", x0=None, rtol=1e-8):
    """Velocity parity for systems where CG amplifies rounding: within 1e-8 of
    the oracle, or within 10x the spread between the oracle and a second CPU
    implementation at the same iteration count (both correct FP64 runs of the
    same recurrence in different summation orders).  Iteration counts may
    differ by more than one where the residual creeps along the tolerance:
    then the oracle's own recurrence residual at the GPU's count must be
    within 2x the tolerance (both stopped at the tolerance up to rounding),
    and the comparison is at that count.  Returns (error, spread)."""
    from oracle import oracle as O
    xo, io = O.pcg(A, F, prec, factor, x0=x0)
    if io.iters != iters_gpu:
        xo, io = O.pcg(A, F, prec, factor, x0=x0, fixed_iters=iters_gpu)
        assert io.relres_rec <= 2 * rtol, (iters_gpu, io.relres_rec)
    den = max(np.linalg.norm(xo), 1e-300)
    err = np.linalg.norm(v_gpu - xo) / den
    if err <= 1e-8:
        return err, None
    x2 = second_cpu_pcg(A, F, prec, factor, iters_gpu, x0=x0)
    spread = np.linalg.norm(x2 - xo) / den
    assert err <= 10 * spread, (err, spread)
    return err, spread
