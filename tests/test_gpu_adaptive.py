"""GPU parity of the adaptive minSR step (minsr_step_adaptive): the
lambda = c ||T||_F^(2/3) schedule (Sec. 3.3), the trust-region rate
eta* = eta / ||tau|| (App. F) and the Levenberg-Marquardt damping from the
ratio of measured to predicted decrease (App. G), against the FP64 oracle,
and the report of the step."""
import numpy as np
import pytest
import torch

from oracle import adaptive as oadapt
from oracle import hamiltonian as oham
from tests.gpu_common import gpu, make_pair, need_gpu, rel_err, scaled_theta, to_dev

pytestmark = gpu


@pytest.fixture(autouse=True)
def _gpu():
    need_gpu()


def _gpu_ham(h):
    import paper_2608_18065_amd as pm
    return pm.hamiltonian(h.kind, J=h.J, h=h.h, J2=h.J2, pbc=h.pbc)


def _report(o):
    import paper_2608_18065_amd as pm
    return dict(zip(pm.ADAPT_REPORT, o["report"].cpu().numpy().tolist()))


def _close(a, b, tol):
    return abs(a - b) <= tol * max(abs(b), 1e-300)


def test_const_mode_equals_minsr_step():
    # CONST shift, no trust region: the same iteration as minsr_step, bit for
    # bit, plus the report (||T||_F, the shift, ||e' - lambda x||, e'^T tau)
    import paper_2608_18065_amd as pm
    Ns = 96
    ham = oham.Ham("tfim", J=1.0, h=0.8, pbc=True)
    outs = []
    for adaptive in (False, True):
        spec, m = make_pair(Lx=12, H=16, max_Ns=Ns)
        th = scaled_theta(spec, 50, 1.0)
        m.set_params(to_dev(th))
        mom = torch.zeros(m.Np, dtype=torch.float64, device="cuda")
        if adaptive:
            o = m.step_adaptive(_gpu_ham(ham), Ns, 0.05, 1e-3, 0.4, mom, 21, 2,
                                form=pm.FORM_FP64_REF)
        else:
            o = m.step(_gpu_ham(ham), Ns, 0.05, 1e-3, 0.4, mom, 21, 2, form=pm.FORM_FP64_REF)
        torch.cuda.synchronize()
        outs.append((o, mom.clone(), m.get_params().clone()))
        m.close()
    (a, ma, ta), (b, mb, tb) = outs
    assert int(b["status"].item()) == 0
    assert torch.equal(a["dtheta"], b["dtheta"]) and torch.equal(ma, mb) and torch.equal(ta, tb)
    assert torch.equal(a["lambda_used"], b["lambda_used"]) and torch.equal(a["tnorm"], b["tnorm"])
    ref = oadapt.step(spec, th, np.zeros_like(th), ham, Ns, 0.05, 1e-3, 0.4, 21, 2)
    d = _report(b)
    assert _close(d["tnorm_frob"], ref["tnorm"], 1e-12)
    assert d["lambda"] == 1e-3 and d["eta"] == 0.05
    assert _close(d["tau_norm"], ref["tau_norm"], 1e-10)
    assert _close(d["ep_tau"], ref["ep_tau"], 1e-10)
    assert d["E_trial"] == 0.0 and d["rho"] == 0.0 and d["lambda_next"] == 0.0


@pytest.mark.parametrize("arch,ham,Ns", [
    (dict(Lx=12, H=16), oham.Ham("tfim", J=1.0, h=1.0, pbc=True), 100),
    (dict(Lx=9, H=8, cplx=True), oham.Ham("cluster"), 70),
], ids=["tfim", "cluster_c"])
def test_step_pow23_trust_region_fp64(arch, ham, Ns):
    # lambda = 3e-4 ||T||_F^{2/3} and eta* = eta / ||e' - lambda x||
    import paper_2608_18065_amd as pm
    spec, m = make_pair(**arch, max_Ns=Ns)
    th = scaled_theta(spec, 51, 1.0)
    m.set_params(to_dev(th))
    mom = torch.zeros(m.Np, dtype=torch.float64, device="cuda")
    print("pow23 + trust region %s Ns=%d" % (arch, Ns), flush=True)
    o = m.step_adaptive(_gpu_ham(ham), Ns, 0.05, 3e-4, 0.4, mom, 23, 1, form=pm.FORM_FP64_REF,
                        lambda_mode=pm.LAMBDA_POW23, trust_region=True)
    torch.cuda.synchronize()
    assert int(o["status"].item()) == 0
    ref = oadapt.step(spec, th, np.zeros_like(th), ham, Ns, 0.05, 3e-4, 0.4, 23, 1,
                      lam_mode="pow23", trust_region=True)
    assert np.array_equal(o["sigma"].cpu().numpy(), ref["sigma"].astype(np.uint8))
    d = _report(o)
    assert _close(d["tnorm_frob"], ref["tnorm"], 1e-12)
    assert _close(d["lambda"], ref["lam_used"], 1e-12)
    assert _close(float(o["lambda_used"].item()), ref["lam_used"], 1e-12)
    assert _close(d["tau_norm"], ref["tau_norm"], 1e-10)
    assert _close(d["ep_tau"], ref["ep_tau"], 1e-10)
    assert _close(d["eta"], ref["eta_used"], 1e-10)
    assert rel_err(o["dtheta"].cpu().numpy(), ref["dtheta"]) < 1e-10
    assert rel_err(mom.cpu().numpy(), ref["m"]) < 1e-10
    m.close()


def test_step_lm_damping_three_steps_fp64():
    # App. G over three consecutive steps: the damping carried on the device
    # follows the oracle's (trial energies from fresh samples of
    # theta - dtheta, ratio, omega rule), with the trust-region rate on
    import paper_2608_18065_amd as pm
    Ns = 80
    spec, m = make_pair(Lx=10, H=16, max_Ns=Ns)
    th = scaled_theta(spec, 52, 1.0)
    m.set_params(to_dev(th))
    ham = oham.Ham("tfim", J=1.0, h=0.9, pbc=False)
    mom = torch.zeros(m.Np, dtype=torch.float64, device="cuda")
    lam_dev = torch.tensor([1e-2], dtype=torch.float64, device="cuda")
    th_ref, m_ref, lam_ref = th, np.zeros_like(th), 1e-2
    seen = set()
    for t in range(3):
        print("LM step %d" % t, flush=True)
        o = m.step_adaptive(_gpu_ham(ham), Ns, 0.08, 0.0, 0.3, mom, 31, t,
                            form=pm.FORM_FP64_REF, lambda_mode=pm.LAMBDA_LM, trust_region=True,
                            omega=1.5, damping=lam_dev)
        torch.cuda.synchronize()
        assert int(o["status"].item()) == 0
        ref = oadapt.step(spec, th_ref, m_ref, ham, Ns, 0.08, lam_ref, 0.3, 31, t,
                          lam_mode="lm", trust_region=True, omega=1.5)
        assert np.array_equal(o["sigma"].cpu().numpy(), ref["sigma"].astype(np.uint8))
        d = _report(o)
        assert d["lambda"] == lam_ref
        assert _close(d["E_trial"], ref["E_trial"], 1e-10)
        assert _close(d["rho"], ref["rho"], 1e-8)
        # the rule's branch is decided away from its thresholds
        assert min(abs(ref["rho"] - 0.25), abs(ref["rho"] - 0.75)) > 1e-6
        assert d["lambda_next"] == ref["lam_next"]
        assert float(lam_dev.item()) == ref["lam_next"]
        assert rel_err(o["dtheta"].cpu().numpy(), ref["dtheta"]) < 1e-10
        assert rel_err(mom.cpu().numpy(), ref["m"]) < 1e-10
        assert rel_err(m.get_params().cpu().numpy(), ref["theta"]) < 1e-12
        seen.add(np.sign(np.log(ref["lam_next"] / lam_ref)))
        th_ref, m_ref, lam_ref = ref["theta"], ref["m"], ref["lam_next"]
    print("lambda branches taken:", sorted(seen))
    m.close()


def test_step_pinv_trust_region_fp64():
    # pseudo-inverse step (lambda = 0, App. F) with tau = T x: the rate and
    # dtheta against the oracle within the pseudo-inverse's tolerance
    import paper_2608_18065_amd as pm
    Ns, cutoff = 120, 1e-8
    spec, m = make_pair(Lx=4, Ly=4, dim=2, H=16, marshall=True, zero_mag=True, max_Ns=Ns)
    th = scaled_theta(spec, 31, 1.0)
    m.set_params(to_dev(th))
    ham = oham.Ham("j1j2", J=1.0)
    mom = torch.zeros(m.Np, dtype=torch.float64, device="cuda")
    o = m.step_adaptive(_gpu_ham(ham), Ns, 0.05, 0.0, 0.0, mom, 8, 3, form=pm.FORM_FP64_REF,
                        pinv_cutoff=cutoff, trust_region=True)
    torch.cuda.synchronize()
    assert int(o["status"].item()) == 0
    ref = oadapt.step(spec, th, np.zeros_like(th), ham, Ns, 0.05, 0.0, 0.0, 8, 3,
                      pinv_cutoff=cutoff, trust_region=True)
    assert np.array_equal(o["sigma"].cpu().numpy(), ref["sigma"].astype(np.uint8))
    w = np.linalg.eigvalsh(ref["T"])
    thr = cutoff * w.max()
    assert np.all(np.abs(w - thr) > 1e-6 * thr)
    kept = w[w > thr]
    tol = max(1e-10, 4.0 * Ns * np.finfo(float).eps * w.max() / kept.min())
    d = _report(o)
    assert d["lambda"] == 0.0
    assert _close(d["tnorm_frob"], ref["tnorm"], 1e-12)
    assert _close(d["tau_norm"], ref["tau_norm"], tol)
    g = o["dtheta"].cpu().numpy()
    assert np.linalg.norm(g - ref["dtheta"]) / np.linalg.norm(ref["dtheta"]) < tol
    # the step saturates the trust region: ||O'^T dtheta|| = eta
    v = ref["Op"].T @ g
    assert _close(float(v @ v), 0.05 ** 2, 10 * tol)
    m.close()


def test_bf16_pow23_on_the_benchmark_system():
    # the tfim64 system in the BF16 + FP64 form with the schedule and the
    # trust region: ||T||_F, the shift and tau of the GPU's own T, x and e'
    import paper_2608_18065_amd as pm
    from workloads import WORKLOADS
    wl = WORKLOADS["tfim64"]
    ham = pm.hamiltonian("tfim", J=wl.J, h=wl.h, pbc=wl.pbc)
    spec, m = make_pair(Lx=wl.Lx, H=wl.H, dtype="f32", seed=wl.seed, max_Ns=wl.Ns)
    mom = torch.zeros(m.Np, dtype=torch.float64, device="cuda")
    o = m.step_adaptive(ham, wl.Ns, wl.eta, 3e-4, wl.mu, mom, wl.key, 0,
                        form=pm.FORM_BF16_FP64, lambda_mode=pm.LAMBDA_POW23, trust_region=True)
    torch.cuda.synchronize()
    st = int(o["status"].item())
    assert st & pm.ST_ERRORS == 0
    it = m.intermediates(pm.FORM_BF16_FP64)
    T = it["T"].cpu().numpy()
    d = _report(o)
    tn = float(np.sqrt(np.sum(T * T)))
    assert _close(d["tnorm_frob"], tn, 1e-12)
    lam = 3e-4 * tn ** (2.0 / 3.0)
    floor = 2.0 ** -24 * float(np.trace(T))
    assert _close(d["lambda"], max(lam, floor), 1e-12)
    assert bool(st & pm.ST_SHIFT_FLOOR) == (floor > lam)
    # x on the device is the solution scaled by eta* / eta
    x = it["x"].cpu().numpy() * wl.eta / d["eta"]
    ep = it["eps_prime"].cpu().numpy()
    xs = np.linalg.solve(T + d["lambda"] * np.eye(T.shape[0]), ep)
    assert np.linalg.norm(x - xs) / np.linalg.norm(xs) < 1e-8
    tau = ep - d["lambda"] * xs
    assert _close(d["tau_norm"], float(np.linalg.norm(tau)), 1e-8)
    assert _close(d["eta"], wl.eta / float(np.linalg.norm(tau)), 1e-8)
    print("tfim64 pow23: ||T||_F %.4e lambda %.4e eta* %.4e" % (tn, d["lambda"], d["eta"]))
    m.close()


def test_fp32_form_const_report():
    # FP32 plain form: ||T||_F of its FP32 Gram in the report
    import paper_2608_18065_amd as pm
    Ns = 96
    spec, m = make_pair(Lx=12, H=32, dtype="f32", max_Ns=Ns)
    mom = torch.zeros(m.Np, dtype=torch.float64, device="cuda")
    ham = pm.hamiltonian("tfim", J=1.0, h=1.0, pbc=True)
    o = m.step_adaptive(ham, Ns, 0.05, 1e-3, 0.0, mom, 4, 4, form=pm.FORM_FP32_PLAIN,
                        trust_region=True)
    torch.cuda.synchronize()
    assert int(o["status"].item()) & pm.ST_ERRORS == 0
    T = m.intermediates(pm.FORM_FP32_PLAIN)["T"].double().cpu().numpy()
    d = _report(o)
    assert _close(d["tnorm_frob"], float(np.sqrt(np.sum(T * T))), 1e-12)
    assert d["lambda"] == 1e-3
    m.close()


def test_adaptive_step_rejects_bad_configs():
    import paper_2608_18065_amd as pm
    spec, m = make_pair(Lx=8, H=8, max_Ns=32)
    mom = torch.zeros(m.Np, dtype=torch.float64, device="cuda")
    ham = pm.hamiltonian("tfim")
    with pytest.raises(pm.MinsrError):   # LM without a damping state
        m.step_adaptive(ham, 32, 0.1, 0.0, 0.0, mom, 1, 0, lambda_mode=pm.LAMBDA_LM)
    lam = torch.tensor([1e-2], dtype=torch.float64, device="cuda")
    with pytest.raises(pm.MinsrError):   # omega must exceed 1
        m.step_adaptive(ham, 32, 0.1, 0.0, 0.0, mom, 1, 0, lambda_mode=pm.LAMBDA_LM,
                        damping=lam, omega=1.0)
    with pytest.raises(pm.MinsrError):   # pseudo-inverse takes a constant lambda = 0
        m.step_adaptive(ham, 32, 0.1, 3e-4, 0.0, mom, 1, 0, lambda_mode=pm.LAMBDA_POW23,
                        pinv_cutoff=1e-8)
    with pytest.raises(pm.MinsrError):   # unknown mode
        m.step_adaptive(ham, 32, 0.1, 1e-3, 0.0, mom, 1, 0, lambda_mode=7)
    with pytest.raises(pm.MinsrError):   # an adaptive shift needs an FP64 solve
        m.step_adaptive(ham, 32, 0.1, 3e-4, 0.0, mom, 1, 0, form=pm.FORM_FP32_PLAIN,
                        lambda_mode=pm.LAMBDA_POW23)
    m.close()
