"""The hand-written reverse pass against finite differences and the
oracle, through the C ABI and through torch.autograd."""
import numpy as np
import pytest
import torch

from oracle import jacobian as ojac
from oracle import model as omodel
from oracle import philox
from tests.gpu_common import gpu, make_pair, need_gpu, rel_err, scaled_theta, to_dev

pytestmark = gpu


@pytest.fixture(autouse=True)
def _gpu():
    need_gpu()


def test_cluster_chain_jacobian_fd_checkpointed():
    # the 100-site cluster chain with a d_h = 128 complex-head GRU
    # (50948 parameters), checkpoints every 10 sites, FP64: rows against
    # central differences (eps = 1e-6) of log Psi on a random parameter
    # subset, and against the oracle's reverse pass
    spec, m = make_pair(Lx=100, H=128, cplx=True, seed=2003, max_Ns=8)
    assert m.Np == 50948
    th = omodel.glorot_init(spec, 2003)
    Ns = 4
    sig, _ = m.sample(Ns, key=1003, counter=0)
    O, _ = m.jacobian(sig, ckpt_every=10)
    O = O.cpu().numpy() * np.sqrt(Ns)          # undo the 1/sqrt(Ns) scaling
    D = np.concatenate([O[:Ns], O[Ns:]], axis=0)
    # finite differences through the GPU evaluation
    rng = np.random.default_rng(3)
    ks = rng.choice(m.Np, size=48, replace=False)
    eps = 1e-6
    th_d = to_dev(th)
    for k in ks:
        tp = th_d.clone(); tp[k] += eps
        tm = th_d.clone(); tm[k] -= eps
        m.set_params(tp); lp = m.logpsi(sig).cpu().numpy()
        m.set_params(tm); lm = m.logpsi(sig).cpu().numpy()
        fd = (lp - lm) / (2 * eps)
        got = D[:Ns, k] + 1j * D[Ns:, k]
        assert np.max(np.abs(got - fd)) < 1e-7 * max(1.0, np.max(np.abs(fd))), k
    m.set_params(th_d)
    # oracle reverse pass on two of the samples
    s2 = sig[:2].cpu().numpy()
    Dref = ojac.log_derivatives(spec, th, s2)
    O2, _ = m.jacobian(sig[:2], ckpt_every=10)
    O2 = O2.cpu().numpy() * np.sqrt(2)
    assert rel_err(O2[:2] + 1j * O2[2:], Dref) < 1e-10


def test_autograd_function_gradcheck():
    from paper_2608_18065_amd.autograd import LogPsi
    spec, m = make_pair(Lx=6, H=8, cplx=True, max_Ns=8)
    th = to_dev(scaled_theta(spec, 21, 1.0)).requires_grad_(True)
    sig, _ = m.sample(5, key=1, counter=2)
    assert torch.autograd.gradcheck(lambda t: LogPsi.apply(t, m, sig), (th,), eps=1e-6,
                                    atol=1e-7, rtol=1e-6)


def test_autograd_matches_oracle_vjp():
    from paper_2608_18065_amd.autograd import log_psi
    spec, m = make_pair(Lx=4, Ly=3, dim=2, H=16, cplx=True, marshall=True, max_Ns=16)
    th_np = scaled_theta(spec, 22, 1.0)
    th = to_dev(th_np).requires_grad_(True)
    sig_np, _ = omodel.sample(spec, th_np, philox.uniforms(4, 4, 9, spec.N))
    sig = to_dev(sig_np.astype(np.uint8))
    out = log_psi(th, m, sig)
    w = torch.randn(9, 2, dtype=torch.float64, device="cuda")
    (out * w).sum().backward()
    D = ojac.log_derivatives(spec, th_np, sig_np)
    wn = w.cpu().numpy()
    ref = wn[:, 0] @ D.real + wn[:, 1] @ D.imag
    assert rel_err(th.grad.cpu().numpy(), ref) < 1e-10
    # the forward matches the oracle's log Psi
    lp = omodel.log_psi(spec, th_np, sig_np)
    assert rel_err(out.detach().cpu().numpy(), np.stack([lp.real, lp.imag], 1)) < 1e-12
