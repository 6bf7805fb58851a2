"""A captured graph of one minSR step, replayed, matches eager steps
bitwise (the Philox counter advances on the device between replays)."""
import numpy as np
import pytest
import torch

from tests.gpu_common import gpu, need_gpu

pytestmark = gpu


@pytest.mark.parametrize("dtype,form", [("f64", 0), ("f32", 1)], ids=["fp64", "bf16_fp64"])
def test_graph_replay_matches_eager(dtype, form):
    need_gpu()
    import paper_2608_18065_amd as pm
    ham = pm.hamiltonian("tfim", J=1.0, h=1.0, pbc=True)
    args = dict(Lx=12, Ly=1, dim=1, hidden=32, dtype=dtype, seed=7, max_Ns=96)
    a = pm.Model(**args)
    b = pm.Model(**args)
    ma = torch.zeros(a.Np, dtype=torch.float64, device="cuda")
    mb = torch.zeros(b.Np, dtype=torch.float64, device="cuda")
    ctr = torch.zeros(1, dtype=torch.int64, device="cuda")
    g, ob = b.capture_step(ham, 96, 0.05, 1e-3, 0.5, mb, 11, ctr, form=form)
    torch.cuda.synchronize()
    for i in range(3):
        oa = a.step(ham, 96, 0.05, 1e-3, 0.5, ma, 11, i, form=form)
        torch.cuda.synchronize()
        # unrelated eager work between replays
        junk = torch.randn(1000, device="cuda").sum()
        g.replay()
        torch.cuda.synchronize()
        assert int(ctr.item()) == i + 1
        for k in ("energy", "dtheta", "status", "eloc", "sigma"):
            assert torch.equal(oa[k], ob[k]), (i, k)
        assert torch.equal(a.get_params(), b.get_params())
        assert torch.equal(ma, mb)
        del junk
