"""The learned warm start over overdamped time steps, at reduced size (20k
cells, 30 training steps, 20 test steps): every solve converges to relres
1e-8, and the trained network's guess (energy-picked against v_prev) needs
fewer CG iterations than the previous-step warm start and has a smaller
Gamma-norm error than the zero start."""
import json

import pytest
import torch

from workloads import sphere_cluster, dynamics_noise

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_2410_04512_amd")
from paper_2410_04512_amd import warmstart as W  # noqa: E402


def test_learned_warm_start_gains():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    ctx = P.Context()
    n = 20000
    c = sphere_cluster(n, 0)
    pos = torch.as_tensor(c["pos"]).cuda()
    R = torch.as_tensor(c["radius"]).cuda()
    res = W.run(ctx, pos, R, dynamics_noise, n_steps=50, n_train=30, epochs=30, lr=3e-3,
                log=lambda s: print(s, flush=True))
    s = W.summary(res)
    print(json.dumps(s), flush=True)
    assert s["all_converged"]
    assert s["max_relres_true"] <= 1.0001e-8
    assert s["mean_iters_learned"] < s["mean_iters_prev"]
    assert s["mean_err_net"] < 1.0
    assert s["net_used"] > 0
    ctx.close()
