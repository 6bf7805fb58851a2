"""Spectrum of T and the conditioning diagnostics of App. E (kappa_2 of
T + lambda I and the digit estimate) on the GPU against the oracle, on
designed spectra and on the Gram of a minSR step."""
import math

import numpy as np
import pytest
import torch

from oracle import conditioning as ocond
from oracle import hamiltonian as oham
from oracle import minsr as ominsr
from tests import inputs
from tests.gpu_common import gpu, make_pair, need_gpu, scaled_theta, to_dev

pytestmark = gpu
EPS64 = 2.0 ** -52


@pytest.fixture(autouse=True)
def _gpu():
    need_gpu()


@pytest.fixture(scope="module")
def model():
    need_gpu()
    import paper_2608_18065_amd as pm
    return pm.Model(16, hidden=16, dtype="f64", seed=1, max_Ns=1100)


def _check(w, cond, T, lam, eps):
    n = T.shape[0]
    ref = ocond.spectrum(T)
    wmax = max(abs(ref[0]), abs(ref[-1]))
    # backward-stable eigensolvers on both sides: each eigenvalue within
    # about n u ||T|| of the exact one
    tol = 4.0 * n * EPS64 * wmax + 1e-300
    assert np.all(np.diff(w) >= 0)
    assert np.max(np.abs(w - ref)) < tol, (np.max(np.abs(w - ref)), tol)
    wmin_r, wmax_r, k_r, d_r = ocond.condition(T, lam, eps)
    assert abs(cond[0] - wmin_r) < tol and abs(cond[1] - wmax_r) < tol
    # kappa: relative error of about tol / (max(w_min, 0) + lambda)
    rk = tol / (max(wmin_r, 0.0) + lam) + 4.0 * n * EPS64
    assert abs(cond[2] - k_r) <= rk * k_r
    assert abs(cond[3] - d_r) <= rk / math.log(10.0) + 1e-12


@pytest.mark.parametrize("n", [1, 2, 17, 64, 65, 333, 1000])
def test_spectrum_designed(model, n):
    rng = np.random.default_rng(300 + n)
    w = inputs.spectrum_loguniform(n, 1e6, rng, zeros=min(2, n - 1))
    T, _ = inputs.psd_matrix(w, seed=400 + n)
    wg, cond, st = model.spectrum(to_dev(T), lam=1e-3, eps=2.0 ** -23)
    torch.cuda.synchronize()
    assert int(st.item()) == 0
    _check(wg.cpu().numpy(), cond.cpu().numpy(), T, 1e-3, 2.0 ** -23)


def test_spectrum_repeated_and_zero_matrix(model):
    n = 120
    w = np.repeat([3.0, 1.0, 1e-4, 0.0], n // 4)
    T, _ = inputs.psd_matrix(w, seed=9)
    wg, cond, st = model.spectrum(to_dev(T), lam=1e-2, eps=EPS64)
    torch.cuda.synchronize()
    assert int(st.item()) == 0
    _check(wg.cpu().numpy(), cond.cpu().numpy(), T, 1e-2, EPS64)
    Z = np.zeros((33, 33))
    wz, cz, st = model.spectrum(to_dev(Z), lam=0.5, eps=EPS64)
    torch.cuda.synchronize()
    assert np.all(wz.cpu().numpy() == 0.0)
    assert cz.cpu().numpy()[2] == 1.0


def test_spectrum_of_a_minsr_gram():
    # the Gram of an FP64 step of the N = 10 chain (centred: one exact
    # zero eigenvalue), its conditioning at the step's lambda
    import paper_2608_18065_amd as pm
    spec, m = make_pair(Lx=10, H=16, max_Ns=64)
    th = scaled_theta(spec, 91, 1.0)
    m.set_params(to_dev(th))
    ham = oham.Ham("tfim", J=1.0, h=1.0)
    mom = torch.zeros(m.Np, dtype=torch.float64, device="cuda")
    m.step(pm.hamiltonian("tfim"), 64, 0.01, 1e-3, 0.0, mom, 1001, 0, form=pm.FORM_FP64_REF,
           apply_update=False)
    torch.cuda.synchronize()
    T = m.intermediates(pm.FORM_FP64_REF)["T"]
    wg, cond, st = m.spectrum(T, lam=1e-3, eps=EPS64)
    torch.cuda.synchronize()
    assert int(st.item()) == 0
    ref = ominsr.step(spec, th, np.zeros_like(th), ham, 64, 0.01, 1e-3, 0.0, 1001, 0)
    _check(wg.cpu().numpy(), cond.cpu().numpy(), ref["T"], 1e-3, EPS64)
    print("kappa_2 %.3e, digits %.2f" % (cond[2].item(), cond[3].item()))
