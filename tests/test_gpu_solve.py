"""The regularised solve alone (Eq. minsrR, App. F) on matrices with
designed spectra, against the oracle's solve."""
import numpy as np
import pytest
import torch

from oracle import minsr as ominsr
from tests.gpu_common import gpu, need_gpu, to_dev
from tests import inputs

pytestmark = gpu

MAX_N = 1100


@pytest.fixture(scope="module")
def model():
    need_gpu()
    import paper_2608_18065_amd as pm
    return pm.Model(16, hidden=16, dtype="f64", seed=1, max_Ns=MAX_N)


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


# Cholesky: forward error <~ cond(T + lambda I) * n * u; with cond <= 1e3 the
# FP64 bar of 1e-10 holds with margin at every n here
@pytest.mark.parametrize("n", [1, 5, 63, 64, 65, 130, 200, 511, 1024, 1100])
def test_cholesky_matches_oracle(model, n):
    rng = np.random.default_rng(n)
    w = inputs.spectrum_loguniform(n, 1e3, rng)
    T, _ = inputs.psd_matrix(w, seed=100 + n)
    b = inputs.rhs(n, seed=n)
    lam = 1e-3
    x, st = model.solve(to_dev(T), to_dev(b), lam=lam)
    torch.cuda.synchronize()
    assert int(st.item()) == 0
    ref = ominsr.solve(T, b, lam)
    assert _rel(x.cpu().numpy(), ref) < 1e-10


def test_cholesky_ill_conditioned(model):
    # a centred Gram is singular; the shift sets cond = (1 + lam) / lam
    n = 700
    rng = np.random.default_rng(5)
    w = inputs.spectrum_loguniform(n, 1e12, rng, zeros=3)
    T, _ = inputs.psd_matrix(w, seed=77)
    b = inputs.rhs(n, seed=3)
    lam = 1e-6
    x, st = model.solve(to_dev(T), to_dev(b), lam=lam)
    torch.cuda.synchronize()
    assert int(st.item()) == 0
    ref = ominsr.solve(T, b, lam)
    # cond ~ 1e6: both sides are within ~cond * n * u of the exact x
    assert _rel(x.cpu().numpy(), ref) < 1e-7


def test_cholesky_reports_indefinite(model):
    n = 150
    w = np.linspace(1.0, 0.1, n)
    w[40] = -0.5
    T, _ = inputs.psd_matrix(w, seed=9)
    x, st = model.solve(to_dev(T), to_dev(inputs.rhs(n, 1)), lam=1e-3)
    torch.cuda.synchronize()
    assert int(st.item()) & 0x2   # MINSR_ST_NOT_PD


def test_cholesky_waits_give_up_with_status():
    # with a limit of one poll, waits between workgroups give up at once: the
    # abort word ends every other wait, the kernels exit and the solve
    # reports MINSR_ST_SOLVE_TIMEOUT (its x is not valid); at the built-in
    # limit the same handle solves correctly again
    import paper_2608_18065_amd as pm
    n = 1024
    m = pm.Model(16, hidden=8, dtype="f64", seed=2, max_Ns=n)
    rng = np.random.default_rng(31)
    T, _ = inputs.psd_matrix(inputs.spectrum_loguniform(n, 1e3, rng), seed=32)
    b = inputs.rhs(n, seed=33)
    m.set_tunable("solve_spin_limit", 1)
    assert m.get_tunable("solve_spin_limit") == 1
    x, st = m.solve(to_dev(T), to_dev(b), lam=1e-3)
    torch.cuda.synchronize()
    assert int(st.item()) & pm.ST_SOLVE_TIMEOUT
    m.set_tunable("solve_spin_limit", 0)
    x, st = m.solve(to_dev(T), to_dev(b), lam=1e-3)
    torch.cuda.synchronize()
    assert int(st.item()) == 0
    assert _rel(x.cpu().numpy(), ominsr.solve(T, b, 1e-3)) < 1e-10
    m.close()


def test_step_with_a_solve_that_gave_up_keeps_theta():
    # a minSR step whose solve gave up leaves theta and the momentum as they
    # were, with the failure in the status word
    import paper_2608_18065_amd as pm
    m = pm.Model(12, hidden=16, dtype="f64", seed=3, max_Ns=256)
    th0 = m.get_params().clone()
    mom = torch.zeros(m.Np, dtype=torch.float64, device="cuda")
    m.set_tunable("solve_spin_limit", 1)
    o = m.step(pm.hamiltonian("tfim", J=1.0, h=1.0), 256, 0.05, 1e-3, 0.5, mom, 5, 0,
               form=pm.FORM_FP64_REF)
    torch.cuda.synchronize()
    assert int(o["status"].item()) & pm.ST_SOLVE_TIMEOUT
    assert torch.equal(m.get_params(), th0) and not bool(mom.any())
    m.close()


def test_solve_rejects_bad_arguments(model):
    import paper_2608_18065_amd as pm
    T = torch.eye(4, dtype=torch.float64, device="cuda")
    b = torch.ones(4, dtype=torch.float64, device="cuda")
    with pytest.raises(pm.MinsrError):
        model.solve(T, b, lam=-1.0)
    with pytest.raises(pm.MinsrError):
        model.solve(T, b, lam=1e-3, pinv_cutoff=1e-8)
    big = torch.eye(MAX_N + 1, dtype=torch.float64, device="cuda")
    with pytest.raises(pm.MinsrError):
        model.solve(big, torch.ones(MAX_N + 1, dtype=torch.float64, device="cuda"), lam=1.0)


# ------------------------------------------------------------ pseudo-inverse
U64 = np.finfo(float).eps


def _pinv_tol(w, cutoff):
    """Forward error bound of a backward-stable eigensolver applied to the
    pseudo-inverse: ~ n u lambda_max / lambda_min(kept) (both sides), with a
    floor at the FP64 bar."""
    kept = w[w > cutoff * w.max()]
    return max(1e-10, 4.0 * len(w) * U64 * w.max() / kept.min())


def _check_gap(w, cutoff, rel=1e-6):
    # no eigenvalue so close to the threshold that rounding could flip its
    # keep/drop decision
    thr = cutoff * w.max()
    assert np.all(np.abs(w - thr) > rel * thr), "ambiguous cutoff in the test input"


@pytest.fixture(scope="module")
def pmodel():
    need_gpu()
    import paper_2608_18065_amd as pm
    return pm.Model(16, hidden=16, dtype="f64", seed=1, max_Ns=MAX_N, pinv=True)


@pytest.mark.parametrize("n", [1, 2, 3, 17, 64, 65, 130, 333, 1000])
def test_pinv_matches_oracle(pmodel, n):
    rng = np.random.default_rng(1000 + n)
    w = inputs.spectrum_loguniform(n, 1e6, rng, zeros=n // 5)
    T, _ = inputs.psd_matrix(w, seed=200 + n)
    b = inputs.rhs(n, seed=n)
    cutoff = 1e-8
    wo = np.linalg.eigvalsh(T)
    _check_gap(wo, cutoff)
    x, st = pmodel.solve(to_dev(T), to_dev(b), lam=0.0, pinv_cutoff=cutoff)
    torch.cuda.synchronize()
    assert int(st.item()) == 0
    ref = ominsr.solve(T, b, 0.0, cutoff)
    assert _rel(x.cpu().numpy(), ref) < _pinv_tol(wo, cutoff)


@pytest.mark.parametrize("n", [40, 257])
def test_pinv_repeated_eigenvalues(pmodel, n):
    # heavily repeated spectrum (deflation by rotations) with an exact null space
    rng = np.random.default_rng(n)
    w = np.round(rng.uniform(0.0, 3.0, n)) * 0.5
    T, _ = inputs.psd_matrix(w, seed=300 + n)
    b = inputs.rhs(n, seed=5)
    x, st = pmodel.solve(to_dev(T), to_dev(b), lam=0.0, pinv_cutoff=1e-8)
    torch.cuda.synchronize()
    assert int(st.item()) == 0
    ref = ominsr.solve(T, b, 0.0, 1e-8)
    assert _rel(x.cpu().numpy(), ref) < 1e-10


def test_pinv_drops_below_cutoff(pmodel):
    # half the spectrum far below the cutoff: x is the solution restricted to
    # the kept eigenvectors, orthogonal to the dropped ones
    n = 300
    rng = np.random.default_rng(11)
    w = np.exp(rng.uniform(np.log(1e-4), 0.0, n))
    w[::2] = 1e-12 * rng.uniform(0.5, 1.0, n)[::2]
    w[1] = 1.0
    T, Q = inputs.psd_matrix(w, seed=12)
    b = inputs.rhs(n, seed=13)
    x, st = pmodel.solve(to_dev(T), to_dev(b), lam=0.0, pinv_cutoff=1e-8)
    torch.cuda.synchronize()
    xh = x.cpu().numpy()
    keep = w > 1e-8 * w.max()
    expect = Q[:, keep] @ ((Q[:, keep].T @ b) / w[keep])
    assert _rel(xh, expect) < 1e-9
    assert np.linalg.norm(Q[:, ~keep].T @ xh) < 1e-9 * np.linalg.norm(xh)


def test_pinv_centred_gram_is_orthogonal_to_ones(pmodel):
    # a centred Gram has T 1 = 0; the pseudo-inverse solution is orthogonal to 1
    n, Np = 200, 500
    rng = np.random.default_rng(21)
    O = rng.standard_normal((n, Np))
    O -= O.mean(axis=0, keepdims=True)
    T = O @ O.T
    T = 0.5 * (T + T.T)
    b = rng.standard_normal(n)
    x, st = pmodel.solve(to_dev(T), to_dev(b), lam=0.0, pinv_cutoff=1e-8)
    torch.cuda.synchronize()
    xh = x.cpu().numpy()
    assert abs(xh.sum()) < 1e-10 * np.sqrt(n) * np.linalg.norm(xh)
    ref = ominsr.solve(T, b, 0.0, 1e-8)
    assert _rel(xh, ref) < _pinv_tol(np.linalg.eigvalsh(T), 1e-8)


def test_pinv_zero_matrix(pmodel):
    n = 70
    T = np.zeros((n, n))
    x, st = pmodel.solve(to_dev(T), to_dev(np.ones(n)), lam=0.0, pinv_cutoff=1e-8)
    torch.cuda.synchronize()
    assert int(st.item()) == 0
    assert float(x.abs().max()) == 0.0


@pytest.mark.parametrize("Ns", [300, 512], ids=["n600_ragged", "n1024"])
def test_fp32_form_solve_matches_its_system(Ns):
    # the FP32 form solves (T + lambda I) x = eps' in FP32 with the same
    # one-launch factorisation (FP32 matrix cores): x against the FP64 oracle
    # solve of the same FP32 T, within the FP32 forward-error bound
    # 4 n u cond(T + lambda I), u = 2^-24
    import paper_2608_18065_amd as pm
    from oracle import hamiltonian as oham
    from tests.gpu_common import make_pair
    spec, m = make_pair(Lx=20, H=32, cplx=True, dtype="f32", max_Ns=Ns)
    ham = pm.hamiltonian("cluster", J=1.0, h=0.0, J2=0.0, pbc=True)
    mom = torch.zeros(m.Np, dtype=torch.float64, device="cuda")
    lam = 0.1
    o = m.step(ham, Ns, 0.01, lam, 0.0, mom, 7, 0, form=pm.FORM_FP32_PLAIN)
    it = m.intermediates(pm.FORM_FP32_PLAIN)
    torch.cuda.synchronize()
    assert int(o["status"].item()) & pm.ST_ERRORS == 0
    T = it["T"].double().cpu().numpy()
    ep = it["eps_prime"].cpu().numpy()
    x = it["x"].cpu().numpy()
    n = T.shape[0]
    ref = ominsr.solve(T, ep, lam)
    kappa = np.linalg.cond(T + lam * np.eye(n))
    err = _rel(x, ref)
    print("FP32 solve n=%d: rel err %.2e, cond %.1e" % (n, err, kappa))
    assert err < 4 * n * 2.0 ** -24 * kappa
