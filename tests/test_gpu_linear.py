"""GPU checks of the linear recurrent test model of App. C through the C ABI
(model option MINSR_OPT_LINEAR): log Psi, samples and log-derivative rows
against the FP64 oracle; the exact gauge zero modes of Prop. 1 in the GPU's
O rows and in its parameter-space metric S at the benchmark's shape (N = 64,
d_h = 64, N_s = 1024); the Gram T of every form against the oracle's O'; and
the closed-form bias element of Prop. 2 in the population S that the GPU's
log-derivatives give over all 2^N configurations."""
import math

import numpy as np
import pytest
import torch

from oracle import linear_rnn as lr
from oracle import philox
from tests import inputs
from tests.gpu_common import gpu, need_gpu, rel_err, to_dev

pytestmark = gpu


@pytest.fixture(autouse=True)
def _gpu():
    need_gpu()


def _model(N, H, max_Ns, theta=None, seed=3):
    import paper_2608_18065_amd as pm
    m = pm.Model(N, 1, 1, H, dtype="f64", seed=seed, max_Ns=max_Ns, linear=True)
    assert m.Np == lr.num_params(H)
    if theta is not None:
        m.set_params(to_dev(theta))
    return m


def _configs(Ns, N, seed):
    return np.random.default_rng(seed).integers(0, 2, size=(Ns, N)).astype(np.int64)


def test_linear_init_blocks():
    H, N = 16, 8
    m = _model(N, H, 4)
    th = m.get_params().cpu().numpy()
    o = lr.offsets(H)
    W, V, b, U, c = lr.unpack(th, H)
    assert np.all(b == 0) and np.all(c == 0)
    for M, (r, cc) in ((W, (H, H)), (V, (H, 2)), (U, (2, H))):
        a = math.sqrt(6.0 / (r + cc))
        assert np.all(np.abs(M) <= a) and np.abs(M).max() > 0.5 * a
    assert o["c"] + 2 == m.Np
    m.close()


@pytest.mark.parametrize("H", [8, 16, 32, 64])
def test_linear_logpsi_and_jacobian_match_oracle(H):
    N, Ns = 12, 40
    th = inputs.linear_theta(H, 100 + H)
    m = _model(N, H, Ns, th)
    sig = _configs(Ns, N, H)
    print("linear H=%d N=%d Ns=%d" % (H, N, Ns), flush=True)
    lp = m.logpsi(to_dev(sig.astype(np.uint8)))
    O, _ = m.jacobian(to_dev(sig.astype(np.uint8)))
    torch.cuda.synchronize()
    lp_ref = lr.log_psi(th, H, sig)
    O_ref = lr.log_derivatives(th, H, sig) / math.sqrt(Ns)
    assert np.all(lp.imag.cpu().numpy() == 0.0)
    assert rel_err(lp.real.cpu().numpy(), lp_ref) < 1e-13
    assert rel_err(O.cpu().numpy(), O_ref) < 1e-12
    m.close()


def test_linear_sampling_matches_oracle():
    H, N, Ns, key, ctr = 16, 20, 64, 77, 5
    th = inputs.linear_theta(H, 7)
    m = _model(N, H, Ns, th)
    u = philox.uniforms(key, ctr, Ns, N)
    ref_sig, ref_lp = lr.sample(th, H, N, u)
    for given in (True, False):
        sig, lp = m.sample(Ns, key=key, counter=ctr, uniforms=to_dev(u) if given else None)
        torch.cuda.synchronize()
        assert np.array_equal(sig.cpu().numpy(), ref_sig.astype(np.uint8)), given
        assert rel_err(lp.real.cpu().numpy(), ref_lp) < 1e-13
    m.close()


@pytest.mark.parametrize("form,tol", [(0, 1e-12), (1, 2e-5), (2, 2e-5), (3, 2e-2)],
                         ids=["fp64", "bf16_fp64", "fp32_plain", "bf16_1pass"])
def test_linear_gram_matches_oracle(form, tol):
    # T = O' O'^T of the centred real form, in each form's arithmetic, against
    # the product of the oracle's O' in FP64 (tolerances: the operand's
    # representation error, 2^-17 for a BF16 hi/lo pair, 2^-24 for FP32,
    # 2^-9 for one BF16, summed over the rows)
    H, N, Ns = 16, 12, 100
    th = inputs.linear_theta(H, 21)
    m = _model(N, H, Ns, th)
    sig = _configs(Ns, N, 22)
    T = m.gram(to_dev(sig.astype(np.uint8)), form=form).cpu().numpy()
    O = lr.log_derivatives(th, H, sig)
    R = (O - O.mean(axis=0)) / math.sqrt(Ns)
    Tref = R @ R.T
    err = float(np.linalg.norm(T - Tref) / np.linalg.norm(Tref))
    print("form %d: ||T - T_ref||_F / ||T_ref||_F = %.2e" % (form, err))
    assert err < tol
    assert np.array_equal(T, T.T)
    m.close()


def test_linear_gauge_zero_modes_full_size():
    # Prop. 1 at the benchmark's shape: every GPU row of O (and of the
    # centred O') annihilates d theta_X to rounding, and so does the GPU's
    # parameter-space metric S; sampled rows agree with the oracle
    H, N, Ns = 64, 64, 1024
    th = inputs.linear_theta(H, 31)
    m = _model(N, H, Ns, th)
    print("linear gauge full size H=%d N=%d Ns=%d" % (H, N, Ns), flush=True)
    sig, _ = m.sample(Ns, key=901, counter=0)
    O, _ = m.jacobian(sig)
    Oc, _ = m.jacobian(sig, centered=True)
    S = m.param_gram(sig)
    torch.cuda.synchronize()
    rng = np.random.default_rng(32)
    for t in range(3):
        X = rng.standard_normal((H, H))
        d = to_dev(lr.gauge_direction(th, H, X))
        for A in (O, Oc):
            v = (A @ d).abs()
            scale = A.abs() @ d.abs()
            worst = float((v / scale).max())
            assert worst < 1e-12, worst
        r = float(torch.linalg.norm(S @ d) / (torch.linalg.norm(S) * torch.linalg.norm(d)))
        assert r < 1e-12, r
    # a generic direction is not a zero mode
    g = torch.randn(m.Np, dtype=torch.float64, device="cuda")
    assert float(torch.linalg.norm(S @ g) / (torch.linalg.norm(S) * torch.linalg.norm(g))) > 1e-6
    # sampled rows against the oracle
    idx = [0, 1, 511, 1023]
    s_np = sig.cpu().numpy().astype(np.int64)[idx]
    ref = lr.log_derivatives(th, H, s_np) / math.sqrt(Ns)
    assert rel_err(O.cpu().numpy()[idx], ref) < 1e-12
    m.close()


@pytest.mark.parametrize("r", [1.0, 1.3])
def test_linear_prop2_closed_form_on_gpu(r):
    # the population S from the GPU's log Psi and O over all 2^N
    # configurations: its bias element along the mode with multiplier r
    # equals (1/4) sum_i m_{i-1}(r)^2 chi_{a,i} (Eq. Sbaba, chi from the
    # oracle by enumeration) and bounds lambda_max(S) from below
    H, N, a = 8, 10, 0
    diag = [r] + [0.5, -0.4, 0.3, 0.2, -0.6, 0.7, 0.1]
    th = inputs.linear_theta(H, 41, diag=diag)
    n = 2 ** N
    m = _model(N, H, n, th)
    allc = lr.all_configs(N)
    sg = to_dev(allc.astype(np.uint8))
    lp = m.logpsi(sg).real
    O, _ = m.jacobian(sg)
    torch.cuda.synchronize()
    P = torch.exp(2.0 * lp)
    assert abs(float(P.sum()) - 1.0) < 1e-13
    O = O * math.sqrt(n)
    X = O - P @ O
    S = (X.T * P) @ X
    k = lr.bias_index(H, a)
    cf = lr.closed_form_Sbb(th, H, N, a)
    print("r=%.2f: S_bb gpu %.12e closed form %.12e" % (r, float(S[k, k]), cf))
    assert abs(float(S[k, k]) - cf) < 1e-11 * cf
    lmax = float(torch.linalg.eigvalsh(S).max())
    assert lmax >= cf * (1 - 1e-12)
    chi = lr.chi(th, H, N, a)
    if r == 1.0:
        assert cf >= chi.min() / 4 * (N - 1) * N * (2 * N - 1) / 6 * (1 - 1e-12)
    else:
        mN = (1 - r ** (N - 1)) / (1 - r)
        assert lmax >= 0.25 * mN * mN * chi[N - 1] * (1 - 1e-12)
    # and the gauge directions are in its kernel
    d = to_dev(lr.gauge_direction(th, H, np.random.default_rng(42).standard_normal((H, H))))
    assert float(torch.linalg.norm(S @ d) / (torch.linalg.norm(S) * torch.linalg.norm(d))) < 1e-12
    m.close()


def test_linear_model_rejects_gru_only_calls():
    import paper_2608_18065_amd as pm
    m = _model(8, 8, 16)
    sig = to_dev(np.zeros((4, 8), dtype=np.uint8))
    with pytest.raises(pm.MinsrError):
        m.local_energy(pm.hamiltonian("tfim", J=1.0, h=1.0), sig, m.logpsi(sig))
    mom = torch.zeros(m.Np, dtype=torch.float64, device="cuda")
    with pytest.raises(pm.MinsrError):
        m.step(pm.hamiltonian("tfim", J=1.0, h=1.0), 8, 0.1, 1e-3, 0.0, mom, 1, 0)
    m.close()
    with pytest.raises(pm.MinsrError):
        pm.Model(8, 1, 1, 8, complex_head=True, dtype="f64", max_Ns=4, linear=True)
    with pytest.raises(pm.MinsrError):
        pm.Model(8, 1, 1, 8, dtype="f32", max_Ns=4, linear=True)
    with pytest.raises(pm.MinsrError):
        pm.Model(8, 1, 1, 128, dtype="f64", max_Ns=4, linear=True)
