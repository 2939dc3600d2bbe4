"""A whole batched step (collide -> assemble -> tree -> factor -> batched PCG)
recorded once and replayed as one hipGraph: every replay bitwise equal to the
eager launches (velocities and solve results), with eager work and
synchronisations between replays; changed inputs refused before launching."""
import numpy as np
import pytest
import torch

from workloads import batched_instance

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_2410_04512_amd")
from tests.gpu_util import to_dev  # noqa: E402


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = P.Context()
    yield c
    c.close()


def _batch(sizes, first_seed=1):
    parts = [batched_instance(first_seed + k, n_override=s) for k, s in enumerate(sizes)]
    off = np.concatenate([[0], np.cumsum([p["pos"].shape[0] for p in parts])]).astype(np.int64)
    cat = lambda key: to_dev(np.concatenate([p[key] for p in parts]))  # noqa: E731
    return off, cat("pos"), cat("radius"), cat("force")


def _eager(ctx, off, pos, R, F, prec):
    g = ctx.collide_batched(off, pos, R)
    A = ctx.assemble_gamma(g)
    if prec == "tree":
        M = ctx.factor_tree(g, ctx.build_tree(g))
    elif prec == "jacobi":
        M = ctx.make_jacobi(A)
    else:
        M = None
    return ctx.pcg_solve_batched(A, M, off, F)


def _replays_match(ctx, S, v, v_ref, infos_ref, off, pos, R, F, prec, times=3):
    for r in range(times):
        v.fill_(float("nan"))
        st, infos = S.replay()
        torch.cuda.synchronize()
        assert st == P.OK
        assert torch.equal(v, v_ref), r
        assert infos == infos_ref, r
        # the program's own eager work between replays
        _eager(ctx, off[:3], pos[:int(off[2])], R[:int(off[2])], F[:int(off[2])], prec)
        torch.cuda.synchronize()


@pytest.mark.parametrize("prec", ["tree", "jacobi", "none"])
def test_step_replay_bitwise_equal_small_batch(ctx, prec):
    sizes = [1000, 300, 2000, 57, 1500, 1, 2]
    off, pos, R, F = _batch(sizes)
    print(f"step: small batch {prec}", flush=True)
    v_ref, infos_ref = _eager(ctx, off, pos, R, F, prec)
    v = torch.zeros_like(F)
    S = P.Step(ctx)
    rec = S.record_batched(off, pos, R, F, v, prec=prec)
    assert rec == infos_ref and torch.equal(v, v_ref)
    values, nbytes = S.size()
    print(f"step: {values} recorded values, {nbytes} bytes", flush=True)
    _replays_match(ctx, S, v, v_ref, infos_ref, off, pos, R, F, prec)


def test_step_replay_refuses_changed_inputs(ctx):
    off, pos, R, F = _batch([800, 1200, 500])
    v_ref, infos_ref = _eager(ctx, off, pos, R, F, "tree")
    v = torch.zeros_like(F)
    S = P.Step(ctx)
    S.record_batched(off, pos, R, F, v)
    F0 = F[5, 1].item()
    F[5, 1] = F0 + 1.0
    v.fill_(7.0)
    st, _ = S.replay(check=False)
    torch.cuda.synchronize()
    assert st == P.ESTALE
    assert torch.all(v == 7.0)     # nothing was launched
    F[5, 1] = F0
    st, infos = S.replay()
    torch.cuda.synchronize()
    assert st == P.OK and torch.equal(v, v_ref) and infos == infos_ref


def test_step_replay_256_batch(ctx):
    """The benchmark's batched workload (256 spheroids, sizes log-uniform in
    [1e3, 2e5], seeds 1..256) with the default knobs."""
    parts = [batched_instance(k + 1) for k in range(256)]
    off = np.concatenate([[0], np.cumsum([p["pos"].shape[0] for p in parts])]).astype(np.int64)
    pos = to_dev(np.concatenate([p["pos"] for p in parts]))
    R = to_dev(np.concatenate([p["radius"] for p in parts]))
    F = to_dev(np.concatenate([p["force"] for p in parts]))
    del parts
    print(f"step: 256 batch, {int(off[-1])} cells: eager", flush=True)
    v_ref, infos_ref = _eager(ctx, off, pos, R, F, "tree")
    v = torch.zeros_like(F)
    S = P.Step(ctx)
    print("step: 256 batch: record", flush=True)
    rec = S.record_batched(off, pos, R, F, v)
    assert rec == infos_ref and torch.equal(v, v_ref)
    assert all(i["status"] == 0 for i in rec)
    for r in range(2):
        print(f"step: 256 batch: replay {r}", flush=True)
        v.fill_(float("nan"))
        st, infos = S.replay()
        torch.cuda.synchronize()
        assert st == P.OK and torch.equal(v, v_ref) and infos == infos_ref
