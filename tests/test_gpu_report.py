"""The step's report of its shift and of the trace norm of T (minsr_step_out
dev_lambda_used, dev_tnorm; the status bit of the BF16 shift floor) against
the oracle's T and the definition max(lambda, 2^-24 tr T)."""
import numpy as np
import pytest
import torch

from oracle import hamiltonian as oham
from oracle import minsr as ominsr
from tests.gpu_common import gpu, make_pair, need_gpu, scaled_theta, to_dev

pytestmark = gpu


@pytest.fixture(autouse=True)
def _gpu():
    need_gpu()


def _gpu_ham(h):
    import paper_2608_18065_amd as pm
    return pm.hamiltonian(h.kind, J=h.J, h=h.h, J2=h.J2, pbc=h.pbc)


def test_report_fp64_form_against_oracle():
    import paper_2608_18065_amd as pm
    spec, m = make_pair(Lx=12, H=16, max_Ns=100)
    th = scaled_theta(spec, 81, 1.0)
    m.set_params(to_dev(th))
    ham = oham.Ham("tfim", J=1.0, h=1.0, pbc=True)
    mom = torch.zeros(m.Np, dtype=torch.float64, device="cuda")
    o = m.step(_gpu_ham(ham), 100, 0.05, 2e-3, 0.0, mom, 3, 5, form=pm.FORM_FP64_REF)
    torch.cuda.synchronize()
    assert int(o["status"].item()) == 0
    ref = ominsr.step(spec, th, np.zeros_like(th), ham, 100, 0.05, 2e-3, 0.0, 3, 5)
    tr = float(np.trace(ref["T"]))
    assert abs(float(o["tnorm"].item()) - tr) < 1e-12 * tr
    assert float(o["lambda_used"].item()) == 2e-3


def test_report_bf16_shift_floor():
    # the benchmark system at its first step: lambda = 1e-3 is above the
    # floor (used as given, no status bit); lambda = 1e-9 is below it (the
    # floor 2^-24 tr T is used, MINSR_ST_SHIFT_FLOOR set, the update applied)
    import paper_2608_18065_amd as pm
    from workloads import WORKLOADS
    wl = WORKLOADS["tfim64"]
    ham = pm.hamiltonian("tfim", J=wl.J, h=wl.h, pbc=wl.pbc)
    for lam in (1e-3, 1e-9):
        spec, m = make_pair(Lx=wl.Lx, H=wl.H, dtype="f32", seed=wl.seed, max_Ns=wl.Ns)
        th0 = m.get_params().clone()
        mom = torch.zeros(m.Np, dtype=torch.float64, device="cuda")
        o = m.step(ham, wl.Ns, wl.eta, lam, 0.0, mom, wl.key, 0, form=pm.FORM_BF16_FP64)
        torch.cuda.synchronize()
        st = int(o["status"].item())
        T = m.intermediates(pm.FORM_BF16_FP64)["T"].cpu().numpy()
        tr = float(np.trace(T))
        floor = 2.0 ** -24 * tr
        assert abs(float(o["tnorm"].item()) - tr) < 1e-12 * tr
        used = float(o["lambda_used"].item())
        if lam > floor:
            assert st == 0 and used == lam
        else:
            assert st == pm.ST_SHIFT_FLOOR
            assert abs(used - floor) <= 1e-15 * floor
        assert not torch.equal(m.get_params(), th0)
        print("lambda %.1e: used %.3e (floor %.3e, tr T %.3e)" % (lam, used, floor, tr))
        m.close()


def test_report_fp32_form_and_pinv():
    import paper_2608_18065_amd as pm
    spec, m = make_pair(Lx=12, H=32, dtype="f32", max_Ns=96)
    mom = torch.zeros(m.Np, dtype=torch.float64, device="cuda")
    o = m.step(pm.hamiltonian("tfim", pbc=True), 96, 0.05, 1e-3, 0.0, mom, 4, 4,
               form=pm.FORM_FP32_PLAIN)
    torch.cuda.synchronize()
    T = m.intermediates(pm.FORM_FP32_PLAIN)["T"].double().cpu().numpy()
    tr = float(np.trace(T))
    assert abs(float(o["tnorm"].item()) - tr) < 1e-12 * tr
    assert float(o["lambda_used"].item()) == 1e-3
    # pseudo-inverse step: shift 0, trace norm of its FP64 T
    spec, m2 = make_pair(Lx=4, Ly=4, dim=2, H=16, marshall=True, zero_mag=True, max_Ns=120)
    mom2 = torch.zeros(m2.Np, dtype=torch.float64, device="cuda")
    o2 = m2.step(pm.hamiltonian("j1j2"), 120, 0.05, 0.0, 0.0, mom2, 8, 3,
                 form=pm.FORM_FP64_REF, pinv_cutoff=1e-8)
    torch.cuda.synchronize()
    assert int(o2["status"].item()) == 0
    T2 = m2.intermediates(pm.FORM_FP64_REF)["T"].cpu().numpy()
    tr2 = float(np.trace(T2))
    assert abs(float(o2["tnorm"].item()) - tr2) < 1e-12 * tr2
    assert float(o2["lambda_used"].item()) == 0.0
