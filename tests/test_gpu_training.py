"""A short training run of the tfim64 workload in the headline BF16 form.

Single steps are checked against the oracle elsewhere; this run checks what
only a trajectory shows: as the log-derivatives grow during training, T + lambda I
must stay numerically positive definite (no step may report a non-positive
pivot or a non-finite update) and the energy must come down.
"""
import sys
import os

import numpy as np
import pytest
import torch

from tests.gpu_common import gpu, need_gpu

pytestmark = gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def test_tfim64_training_steps_stay_positive_definite():
    need_gpu()
    import paper_2608_18065_amd as pm
    from workloads import WORKLOADS
    wl = WORKLOADS["tfim64"]
    ham = pm.hamiltonian(wl.ham, J=wl.J, h=wl.h, pbc=wl.pbc)
    m = pm.Model(wl.Lx, wl.Ly, wl.dim, wl.H, wl.complex_head, wl.marshall, wl.zero_mag,
                 dtype="f32", seed=wl.seed, max_Ns=wl.Ns)
    mom = torch.zeros(m.Np, dtype=torch.float64, device="cuda")
    outs = m.step_outputs(wl.Ns)
    K = 200
    hist = torch.zeros((K, 3), dtype=torch.float64, device="cuda")
    status = torch.zeros(K, dtype=torch.int32, device="cuda")
    for i in range(K):
        m.step(ham, wl.Ns, wl.eta, wl.lam, wl.mu, mom, wl.key, i, form=pm.FORM_BF16_FP64,
               ckpt_every=wl.ckpt_every, outputs=outs)
        hist[i].copy_(outs["energy"])
        status[i:i + 1].copy_(outs["status"])
    torch.cuda.synchronize()
    st = status.cpu().numpy()
    E = hist.cpu().numpy()[:, 0] / (wl.Lx * wl.Ly)
    m.close()
    bad = np.nonzero(st & pm.ST_ERRORS)[0]
    assert len(bad) == 0, "steps with failure bits: %s" % bad[:10]
    print("steps whose shift was raised to the BF16 floor: %d" %
          np.count_nonzero(st & pm.ST_SHIFT_FLOOR))
    # from about 0.25 per site above the ground energy to below 1e-2
    assert E[0] - wl.E0 / 64 > 0.1
    assert E[-20:].mean() - wl.E0 / 64 < 1e-2
