"""The parameter-space metric S = O' O'^T (Eq. SR; the subsampled QGT of
Prop. 3) on the GPU against the oracle, and its spectrum against T's."""
import numpy as np
import pytest
import torch

from oracle import jacobian as ojac
from oracle import model as omodel
from oracle import philox
from oracle import qgt as oqgt
from tests.gpu_common import gpu, make_pair, need_gpu, rel_err, scaled_theta, to_dev

pytestmark = gpu


@pytest.fixture(autouse=True)
def _gpu():
    need_gpu()


@pytest.mark.parametrize("arch,Ns", [
    (dict(Lx=10, H=16), 50),
    (dict(Lx=9, H=8, cplx=True), 70),
    (dict(Lx=6, Ly=6, dim=2, H=8, cplx=True, marshall=True), 130),
], ids=["prnn1d", "crnn1d", "crnn2d_6x6"])
def test_param_gram_fp64(arch, Ns):
    spec, m = make_pair(**arch, max_Ns=Ns)
    th = scaled_theta(spec, 95, 1.0)
    m.set_params(to_dev(th))
    sig, _ = omodel.sample(spec, th, philox.uniforms(31, 2, Ns, spec.N))
    S = m.param_gram(to_dev(sig.astype(np.uint8))).cpu().numpy()
    D = ojac.log_derivatives(spec, th, sig)
    ref = oqgt.subsampled_S(D)
    assert S.shape == (m.Np, m.Np)
    assert np.array_equal(S, S.T)
    assert rel_err(S, ref) < 1e-10


def test_param_gram_fp32_model():
    spec, m = make_pair(Lx=12, H=32, dtype="f32", max_Ns=64)
    th = scaled_theta(spec, 96, 1.0)
    m.set_params(to_dev(th))
    sig, _ = omodel.sample(spec, th, philox.uniforms(32, 2, 64, spec.N))
    S = m.param_gram(to_dev(sig.astype(np.uint8))).cpu().numpy()
    ref = oqgt.subsampled_S(ojac.log_derivatives(spec, th, sig))
    assert rel_err(S, ref) < 1e-4
