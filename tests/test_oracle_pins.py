"""Pins for the FP64 oracle: each check ties an oracle function to
something other than itself (numpy's Philox, enumeration, dense Hamiltonians,
closed forms, finite differences, the push-through identity)."""
import math
import os

import numpy as np
import pytest

from oracle import hamiltonian as ham_mod
from oracle import jacobian, minsr, model, philox
from tests import refs

HERE = os.path.dirname(os.path.abspath(__file__))


def golden(name):
    with open(os.path.join(HERE, "golden", "paper_values.txt")) as f:
        for line in f:
            if line.startswith(name + " "):
                return float(line.split()[1])
    raise KeyError(name)


def scaled_theta(spec, seed, scale):
    """Glorot init with weights scaled up so that conditionals are far from
    uniform (a stronger test than the near-uniform initial state), plus
    non-zero biases."""
    th = model.glorot_init(spec, seed) * scale
    rng = np.random.default_rng(seed)
    off = 0
    for name, shape in model.layout(spec):
        n = int(np.prod(shape))
        if len(shape) == 1:
            th[off:off + n] = rng.uniform(-0.5, 0.5, n)
        off += n
    return th


# --------------------------------------------------------------------- RNG

@pytest.mark.parametrize("key,ctr", [(0, 0), (5, 10), (2**63 + 12345, 2**40 + 7), (2**64 - 1, 2**64 - 2)])
def test_philox_matches_numpy(key, ctr):
    # numpy's Philox (4x64-10) increments its 256-bit counter before each
    # block: its block for counter c is philox4x64(c + 1).
    bg = np.random.Philox(key=np.array([key, 99], dtype=np.uint64),
                          counter=np.array([ctr, 3, 4, 5], dtype=np.uint64))
    raw = bg.random_raw(4)
    c0 = (ctr + 1) % 2**64
    c1 = 3 + (1 if ctr + 1 == 2**64 else 0)
    mine = philox.philox4x64((c0, c1, 4, 5), (key, 99))
    assert [int(x) for x in raw] == list(mine)


def test_uniform_grid():
    u = philox.uniforms(7, 3, 16, 10)
    assert u.shape == (16, 10)
    assert np.all(u >= 0) and np.all(u < 1)
    assert np.all(u * 2.0**53 == np.floor(u * 2.0**53))


# ------------------------------------------------------------ layout/init

@pytest.mark.parametrize("dim,H,cplx,expected", [
    (1, 16, False, 962), (1, 64, False, 13058), (1, 128, False, 50690),
    (1, 128, True, 50948), (2, 128, False, 84226), (2, 128, True, 84484),
    (2, 10, False, 682), (2, 10, True, 704)])
def test_param_counts(dim, H, cplx, expected):
    # App. A cell sizes: 1D 3H^2 + 4*2H + 4H + 2 (+2H+2 for the phase head);
    # 2D adds U1, U2 and doubles the spin input width.
    spec = model.Spec(Lx=4, Ly=4 if dim == 2 else 1, dim=dim, H=H, complex_head=cplx)
    assert model.num_params(spec) == expected


def test_glorot_bounds_and_stats():
    spec = model.Spec(Lx=10, H=64)
    th = model.glorot_init(spec, 2002)
    P = model.unpack(spec, th)
    for name, shape in model.layout(spec):
        if len(shape) == 1:
            assert np.all(P[name] == 0.0)
        else:
            a = math.sqrt(6.0 / (shape[0] + shape[1]))
            w = P[name].ravel()
            assert np.all(np.abs(w) <= a)
            if w.size > 1000:   # uniform(-a, a): mean 0, variance a^2/3
                assert abs(w.mean()) < 0.1 * a
                assert abs(w.var() / (a * a / 3) - 1) < 0.1


def test_path_zigzag():
    spec = model.Spec(Lx=3, Ly=3, dim=2, H=4)
    assert model.path_coords(spec) == [(0, 0), (1, 0), (2, 0), (2, 1), (1, 1), (0, 1), (0, 2), (1, 2), (2, 2)]
    nb = model.neighbours_2d(spec)
    # site (1,1) at k=4: horizontal neighbour (2,1) (k=3), vertical (1,0) (k=1)
    assert nb[4] == (3, 1)
    assert nb[0] == (-1, -1)


# ------------------------------------------------------------ normalisation

SPECS_SMALL = [
    model.Spec(Lx=8, H=6),
    model.Spec(Lx=8, H=6, complex_head=True),
    model.Spec(Lx=3, Ly=3, dim=2, H=5),
    model.Spec(Lx=3, Ly=3, dim=2, H=5, complex_head=True, marshall=True),
]


@pytest.mark.parametrize("spec", SPECS_SMALL)
def test_probabilities_sum_to_one(spec):
    th = scaled_theta(spec, 11, 2.0)
    s = refs.all_configs(spec.N)
    lp = model.log_psi(spec, th, s)
    assert abs(np.sum(np.exp(2 * lp.real)) - 1.0) < 1e-12


def test_zero_mag_mask_normalised_in_sector():
    spec = model.Spec(Lx=4, Ly=2, dim=2, H=5, zero_mag=True, marshall=True)
    th = scaled_theta(spec, 12, 2.0)
    s = refs.all_configs(spec.N)
    P = np.exp(2 * model.log_psi(spec, th, s).real)
    in_sector = s.sum(axis=1) == spec.N // 2
    assert abs(P[in_sector].sum() - 1.0) < 1e-12
    assert np.all(P[~in_sector] == 0.0)


def test_config1_enumeration_normalised():
    spec = model.Spec(Lx=10, H=16)
    th = model.glorot_init(spec, 2001)
    lp = model.log_psi(spec, th, refs.all_configs(10))
    assert abs(np.sum(np.exp(2 * lp.real)) - 1.0) < 1e-12


# ------------------------------------------------------------ sampling

def test_sampling_matches_exact_distribution():
    spec = model.Spec(Lx=5, H=4)
    th = scaled_theta(spec, 3, 3.0)
    u = philox.uniforms(77, 0, 20000, spec.N)
    sig, lp = model.sample(spec, th, u)
    # returned log Psi is the log Psi of the returned configuration
    lp2 = model.log_psi(spec, th, sig)
    assert np.max(np.abs(lp - lp2)) < 1e-13
    allc = refs.all_configs(5)
    P = np.exp(2 * model.log_psi(spec, th, allc).real)
    idx = sig @ (1 << np.arange(4, -1, -1))
    counts = np.bincount(idx, minlength=32)
    expct = P * len(idx)
    chi2 = np.sum((counts - expct) ** 2 / expct)
    # 31 degrees of freedom: chi2 < 70 fails with probability ~1e-4
    assert chi2 < 70.0


def test_sampling_respects_zero_mag():
    spec = model.Spec(Lx=4, Ly=4, dim=2, H=4, zero_mag=True)
    th = scaled_theta(spec, 5, 3.0)
    sig, lp = model.sample(spec, th, philox.uniforms(1, 2, 300, spec.N))
    assert np.all(sig.sum(axis=1) == 8)
    assert np.all(np.isfinite(lp))


# ------------------------------------------------------------ Hamiltonians

def test_tfim_free_fermion_matches_paper_table2():
    e = refs.tfim_obc_free_fermion(200) / 200
    assert abs(e - golden("tfim_obc_N200_exact_E_per_site")) < 5e-11


def test_dense_hamiltonians_exact_energies():
    e = np.linalg.eigvalsh(refs.dense_tfim(10, 1, 1, False))[0]
    assert abs(e - refs.tfim_obc_free_fermion(10)) < 1e-10
    assert abs(e - (-12.381489999654756)) < 1e-10
    e = np.linalg.eigvalsh(refs.dense_tfim(8, 1, 1, True))[0]
    assert abs(e - refs.tfim_pbc_critical(8)) < 1e-10
    e = np.linalg.eigvalsh(refs.dense_cluster_pbc(8))[0]
    assert abs(e / 8 - golden("cluster_exact_E_per_site")) < 1e-12


def _eloc_vs_dense(spec, ham, Hd, seed, scale=2.0):
    th = scaled_theta(spec, seed, scale)
    s = refs.all_configs(spec.N)
    lp = model.log_psi(spec, th, s)
    psi = np.exp(lp)
    eps = ham_mod.local_energy(spec, th, ham, s, lp)
    ok = np.abs(psi) > 0
    ref = (Hd @ psi)[ok] / psi[ok]
    assert np.max(np.abs(eps[ok] - ref)) < 1e-9 * max(1.0, np.max(np.abs(ref)))
    # variational principle for the normalised state
    E = np.sum(np.abs(psi[ok]) ** 2 * eps[ok]).real
    assert E >= np.linalg.eigvalsh(Hd)[0] - 1e-10
    return th


@pytest.mark.parametrize("pbc", [False, True])
def test_eloc_tfim_dense(pbc):
    spec = model.Spec(Lx=8, H=6)
    _eloc_vs_dense(spec, ham_mod.Ham("tfim", J=1.0, h=0.7, pbc=pbc), refs.dense_tfim(8, 1.0, 0.7, pbc), 21)


def test_eloc_cluster_dense_complex():
    spec = model.Spec(Lx=8, H=6, complex_head=True)
    _eloc_vs_dense(spec, ham_mod.Ham("cluster"), refs.dense_cluster_pbc(8), 22)


@pytest.mark.parametrize("J2,cplx", [(0.0, False), (0.5, True)])
def test_eloc_j1j2_dense_marshall(J2, cplx):
    spec = model.Spec(Lx=3, Ly=3, dim=2, H=5, complex_head=cplx, marshall=True)
    _eloc_vs_dense(spec, ham_mod.Ham("j1j2", J=1.0, J2=J2), refs.dense_j1j2(3, 3, 1.0, J2), 23)


def test_eloc_j1j2_dense_zero_mag():
    spec = model.Spec(Lx=4, Ly=2, dim=2, H=5, marshall=True, zero_mag=True)
    _eloc_vs_dense(spec, ham_mod.Ham("j1j2", J=1.0, J2=0.0), refs.dense_j1j2(4, 2, 1.0, 0.0), 24)


def test_eloc_product_state_closed_form():
    # U = 0, c = 0: every conditional is (1/2, 1/2), Psi uniform, so the
    # off-diagonal TFIM ratios are all 1: eps = -J sum zz - h N exactly.
    spec = model.Spec(Lx=10, H=16)
    th = model.glorot_init(spec, 2001)
    P = model.unpack(spec, th)
    P["U"][:] = 0.0
    P["c"][:] = 0.0
    s = refs.all_configs(10)[::7]
    eps = ham_mod.local_energy(spec, th, ham_mod.Ham("tfim", J=1.0, h=1.0), s)
    z = 1 - 2 * s
    expect = -np.sum(z[:, :-1] * z[:, 1:], axis=1) - 10.0
    assert np.all(eps == expect)


def test_marshall_makes_heisenberg_ground_state_positive():
    # With the Marshall sign (-1)^{sigma_A}, the Heisenberg ground state
    # times the sign is non-negative: the sign structure the oracle applies
    # is the exact one at J2 = 0.
    spec = model.Spec(Lx=3, Ly=2, dim=2, H=3, marshall=True)
    Hd = refs.dense_j1j2(3, 2, 1.0, 0.0)
    w, V = np.linalg.eigh(Hd)
    v = V[:, 0]
    s = refs.all_configs(6)
    sign = np.exp(1j * model.marshall_phase(spec, s)).real
    w2 = (v * sign)
    w2 = w2 / w2[np.argmax(np.abs(w2))]
    assert np.min(w2.real) > -1e-10


# ------------------------------------------------------------ Jacobian

def _fd_check(spec, seed, ns=3, h=1e-6):
    th = scaled_theta(spec, seed, 1.5)
    u = philox.uniforms(seed, 0, ns, spec.N)
    sig, _ = model.sample(spec, th, u)
    D = jacobian.log_derivatives(spec, th, sig)
    Dfd = np.zeros_like(D)
    for k in range(th.size):
        tp = th.copy(); tp[k] += h
        tm = th.copy(); tm[k] -= h
        Dfd[:, k] = (model.log_psi(spec, tp, sig) - model.log_psi(spec, tm, sig)) / (2 * h) \
            if np.iscomplexobj(D) else \
            (model.log_psi(spec, tp, sig).real - model.log_psi(spec, tm, sig).real) / (2 * h)
    assert np.max(np.abs(D - Dfd)) < 1e-7 * max(1.0, np.max(np.abs(D)))


@pytest.mark.parametrize("spec", [
    model.Spec(Lx=6, H=4),
    model.Spec(Lx=6, H=4, complex_head=True),
    model.Spec(Lx=3, Ly=3, dim=2, H=3, marshall=True),
    model.Spec(Lx=3, Ly=2, dim=2, H=3, complex_head=True, marshall=True),
    model.Spec(Lx=2, Ly=4, dim=2, H=3, zero_mag=True),
])
def test_jacobian_central_fd(spec):
    _fd_check(spec, 31)


@pytest.mark.parametrize("spec", [model.Spec(Lx=7, H=5), model.Spec(Lx=7, H=5, complex_head=True)])
def test_score_has_zero_mean(spec):
    # sum_sigma P(sigma) d log Psi = 0 for the real part (normalised P); the
    # phase derivative has no such constraint.
    th = scaled_theta(spec, 41, 2.0)
    s = refs.all_configs(spec.N)
    P = np.exp(2 * model.log_psi(spec, th, s).real)
    D = jacobian.log_derivatives(spec, th, s)
    assert np.max(np.abs(P @ D.real)) < 1e-12
    if spec.complex_head:
        assert np.max(np.abs(P @ D.imag)) > 1e-3


@pytest.mark.parametrize("spec,ham,Hd", [
    (model.Spec(Lx=6, H=4), ham_mod.Ham("tfim", J=1.0, h=0.8, pbc=True), refs.dense_tfim(6, 1.0, 0.8, True)),
    (model.Spec(Lx=6, H=4, complex_head=True), ham_mod.Ham("cluster"), refs.dense_cluster_pbc(6)),
])
def test_energy_gradient_by_enumeration(spec, ham, Hd):
    # d<H>/dtheta from central differences of the exactly enumerated energy
    # equals 2 Re sum_sigma P (d log Psi)^* (eps - <H>)  (Sec. 2.3).
    th = scaled_theta(spec, 51, 1.5)
    s = refs.all_configs(spec.N)

    def energy(t):
        psi = np.exp(model.log_psi(spec, t, s))
        return (np.conj(psi) @ (Hd @ psi)).real

    lp = model.log_psi(spec, th, s)
    P = np.exp(2 * lp.real)
    eps = ham_mod.local_energy(spec, th, ham, s, lp)
    E = P @ eps
    D = jacobian.log_derivatives(spec, th, s)
    grad = 2 * np.real(np.conj(D).T @ (P * (eps - E)))
    h = 1e-6
    for k in range(0, th.size, 7):
        tp = th.copy(); tp[k] += h
        tm = th.copy(); tm[k] -= h
        fd = (energy(tp) - energy(tm)) / (2 * h)
        assert abs(fd - grad[k]) < 1e-7 * max(1.0, abs(grad[k]))


# ------------------------------------------------------------ minSR algebra

def _config1_inputs(cplx=False, ns=64):
    spec = model.Spec(Lx=10, H=16, complex_head=cplx)
    th = scaled_theta(spec, 2001, 1.0)
    sig, lp = model.sample(spec, th, philox.uniforms(1001, 0, ns, 10))
    ham = ham_mod.Ham("tfim", J=1.0, h=1.0) if not cplx else ham_mod.Ham("cluster")
    eps = ham_mod.local_energy(spec, th, ham, sig, lp)
    D = jacobian.log_derivatives(spec, th, sig)
    return spec, th, D, eps


@pytest.mark.parametrize("cplx", [False, True])
def test_T_symmetric_psd_and_centred(cplx):
    _, _, D, eps = _config1_inputs(cplx)
    r = minsr.update(D, eps, 0.01, 1e-3)
    T = r["T"]
    n = T.shape[0]
    assert n == (128 if cplx else 64)
    assert np.max(np.abs(T - T.T)) == 0.0
    w = np.linalg.eigvalsh(T)
    assert w[0] > -n * 1e-15 * w[-1]
    ones = np.ones(64)
    for blk in range(n // 64):
        v = np.zeros(n); v[blk * 64:(blk + 1) * 64] = ones
        assert np.max(np.abs(T @ v)) < 1e-12 * w[-1]
    # T and S = O' O'^T share their non-zero spectrum (App. E)
    S = r["Op"] @ r["Op"].T
    ws = np.linalg.eigvalsh(S)[-n:]
    big = w > 1e-8 * w[-1]
    assert np.allclose(np.sort(ws)[-big.sum():], w[big], rtol=1e-9, atol=1e-12 * w[-1])


@pytest.mark.parametrize("cplx", [False, True])
def test_push_through_identity(cplx):
    # minSR (sample space) equals SR (parameter space): Eq. SR vs Eq. minsrR.
    _, _, D, eps = _config1_inputs(cplx)
    eta, lam = 0.01, 1e-3
    r = minsr.update(D, eps, eta, lam)
    Op, ep = r["Op"], r["ep"]
    S = Op @ Op.T
    sr = eta * np.linalg.solve(S + lam * np.eye(S.shape[0]), Op @ ep)
    assert np.max(np.abs(sr - r["dtheta"])) < 1e-9 * np.max(np.abs(sr))


def test_sgd_limit():
    # lambda >> ||S||: dtheta -> (eta/lambda) * 2 Re[Obar ebar], the
    # centred SGD step of Eq. SGD_update, here written from D and eps.
    _, _, D, eps = _config1_inputs(True)
    eta, lam = 0.01, 1e9
    r = minsr.update(D, eps, eta, lam)
    Ns = D.shape[0]
    grad = 2 * np.real((D - D.mean(axis=0)).T @ np.conj(eps - eps.mean())) / Ns
    assert np.max(np.abs(r["dtheta"] * lam / eta - grad)) < 1e-6 * np.max(np.abs(grad))


def test_pseudo_inverse_branch():
    _, _, D, eps = _config1_inputs(False)
    r = minsr.update(D, eps, 1.0, 0.0, pinv_cutoff=1e-8)
    T = r["T"]
    x_ref = np.linalg.pinv(T, rcond=1e-8, hermitian=True) @ r["ep"]
    assert np.max(np.abs(r["x"] - x_ref)) < 1e-8 * np.max(np.abs(x_ref))
    assert abs(np.sum(r["x"])) < 1e-8 * np.max(np.abs(r["x"]))


def test_full_step_config1():
    spec = model.Spec(Lx=10, H=16)
    th = model.glorot_init(spec, 2001)
    res = minsr.step(spec, th, np.zeros_like(th), ham_mod.Ham("tfim"), 64, 0.01, 1e-3, 0.0, 1001, 0)
    assert np.all(np.isfinite(res["dtheta"]))
    assert np.array_equal(res["theta"], th - res["dtheta"])
    # the energy estimate lies above the exact ground energy by a margin
    # far larger than its statistical error at initialisation
    assert res["E"].real > -12.381489999654756


# ------------------------------------------------------------ cell formulas

def _torch_cell_from_paper(P, H, ds):
    """torch.nn.GRUCell whose output equals the App. A cell: torch's update
    gate z plays the role of 1 - u (so its pre-activation is -W_u x - b_u),
    its reset gate is r, and its candidate is tanh(W_in x + b_in +
    r * (W_h h + b_h))."""
    import torch
    cell = torch.nn.GRUCell(ds, H, bias=True).double()
    Wu, Wr = P["Wu"], P["Wr"]
    w_ih = np.concatenate([Wr[:, H:], -Wu[:, H:], P["Win"]], axis=0)
    w_hh = np.concatenate([Wr[:, :H], -Wu[:, :H], P["Wh"]], axis=0)
    b_ih = np.concatenate([P["br"], -P["bu"], P["bin"]])
    b_hh = np.concatenate([np.zeros(H), np.zeros(H), P["bh"]])
    with torch.no_grad():
        cell.weight_ih.copy_(torch.from_numpy(w_ih))
        cell.weight_hh.copy_(torch.from_numpy(w_hh))
        cell.bias_ih.copy_(torch.from_numpy(b_ih))
        cell.bias_hh.copy_(torch.from_numpy(b_hh))
    return cell


@pytest.mark.parametrize("dim", [1, 2])
def test_gru_cell_matches_torch_grucell(dim):
    import torch
    spec = model.Spec(Lx=4, Ly=4 if dim == 2 else 1, dim=dim, H=7)
    th = scaled_theta(spec, 61, 2.0)
    P = model.unpack(spec, th)
    ds = 2 if dim == 1 else 4
    rng = np.random.default_rng(0)
    hprev = rng.normal(size=(9, 7))
    xs = rng.integers(0, 2, size=(9, ds)).astype(float)
    h, _ = model.gru_cell(P, hprev, xs)
    cell = _torch_cell_from_paper(P, 7, ds)
    with torch.no_grad():
        ref = cell(torch.from_numpy(xs), torch.from_numpy(hprev)).numpy()
    assert np.max(np.abs(h - ref)) < 1e-14


def test_1d_log_p_matches_torch_recurrence():
    # whole 1D recurrence: torch GRUCell + log_softmax head, zero initial
    # state and zero first input (Sec. 2, vanilla-cell paragraph)
    import torch
    spec = model.Spec(Lx=9, H=6)
    th = scaled_theta(spec, 62, 2.0)
    P = model.unpack(spec, th)
    cell = _torch_cell_from_paper(P, 6, 2)
    sig = refs.all_configs(9)[::5]
    with torch.no_grad():
        h = torch.zeros(len(sig), 6, dtype=torch.float64)
        x = torch.zeros(len(sig), 2, dtype=torch.float64)
        tot = torch.zeros(len(sig), dtype=torch.float64)
        for k in range(9):
            h = cell(x, h)
            z = h @ torch.from_numpy(P["U"]).T + torch.from_numpy(P["c"])
            lsm = torch.log_softmax(z, dim=1)
            s = torch.from_numpy(sig[:, k])
            tot += lsm[torch.arange(len(sig)), s]
            x = torch.nn.functional.one_hot(s, 2).double()
    lp = model.log_psi(spec, th, sig)
    assert np.max(np.abs(2 * lp.real - tot.numpy())) < 1e-12


def test_head_closed_forms():
    # U = 0, U_phi = 0: conditionals are softmax(c) and phases
    # pi*softsign(c_phi) at every site, independent of the history.
    spec = model.Spec(Lx=6, H=4, complex_head=True)
    th = scaled_theta(spec, 63, 1.0)
    P = model.unpack(spec, th)
    P["U"][:] = 0.0
    P["Uphi"][:] = 0.0
    P["c"][:] = [0.3, -1.1]
    P["cphi"][:] = [0.7, -2.0]
    s = refs.all_configs(6)
    lp = model.log_psi(spec, th, s)
    n0 = np.sum(s == 0, axis=1)
    n1 = 6 - n0
    lse = np.log(np.exp(0.3) + np.exp(-1.1))
    assert np.allclose(2 * lp.real, n0 * (0.3 - lse) + n1 * (-1.1 - lse), rtol=0, atol=1e-13)
    ph = n0 * math.pi * 0.7 / 1.7 + n1 * math.pi * (-2.0) / 3.0
    assert np.allclose(lp.imag, ph, rtol=0, atol=1e-13)


def test_2d_log_p_matches_torch_recurrence():
    # whole 2D recurrence (App. A, 2D cell; Sec. 2.1 zigzag path): torch
    # GRUCell with h' = U1 h(i - (-1)^j, j) + U2 h(i, j - 1) and
    # sigma' = [sigma(i - (-1)^j, j); sigma(i, j - 1)], zero states and zero
    # one-hots outside the lattice.  The path, the neighbour coordinates and
    # the hidden-state grid are built here from the paper's formulas, not
    # from the oracle's path helpers; U1 and U2 are made very different so a
    # swap (or a swapped sigma' order) shows.
    import torch
    Lx, Ly, H = 3, 4, 5
    spec = model.Spec(Lx=Lx, Ly=Ly, dim=2, H=H)
    th = scaled_theta(spec, 64, 2.0)
    P = model.unpack(spec, th)
    P["U1"][:] *= 3.0
    P["U2"][:] *= 0.2
    P["Wu"][:, H:H + 2] += 1.5      # horizontal spin columns differ from vertical
    P["Win"][:, 0:2] -= 1.0
    cell = _torch_cell_from_paper(P, H, 4)
    U1, U2 = torch.from_numpy(P["U1"]), torch.from_numpy(P["U2"])
    U, c = torch.from_numpy(P["U"]), torch.from_numpy(P["c"])
    sig = refs.all_configs(Lx * Ly)[::97]
    ns = len(sig)
    order = []                                  # pi(k) = (i_k, j_k)
    for k in range(Lx * Ly):
        j = k // Lx
        order.append((k % Lx if j % 2 == 0 else Lx - 1 - k % Lx, j))
    pos = {ij: k for k, ij in enumerate(order)}
    with torch.no_grad():
        hgrid = {}
        tot = torch.zeros(ns, dtype=torch.float64)
        for k, (i, j) in enumerate(order):
            ih = i - (1 if j % 2 == 0 else -1)
            h_h = hgrid.get((ih, j), torch.zeros(ns, H, dtype=torch.float64))
            h_v = hgrid.get((i, j - 1), torch.zeros(ns, H, dtype=torch.float64))

            def onehot(ij):
                if ij not in pos:
                    return torch.zeros(ns, 2, dtype=torch.float64)
                return torch.nn.functional.one_hot(torch.from_numpy(sig[:, pos[ij]]), 2).double()
            x = torch.cat([onehot((ih, j)), onehot((i, j - 1))], dim=1)
            hp = h_h @ U1.T + h_v @ U2.T
            h = cell(x, hp)
            hgrid[(i, j)] = h
            lsm = torch.log_softmax(h @ U.T + c, dim=1)
            tot += lsm[torch.arange(ns), torch.from_numpy(sig[:, k])]
    lp = model.log_psi(spec, th, sig)
    ref = tot.numpy()
    assert np.max(np.abs(2 * lp.real - ref)) < 1e-13 * np.max(np.abs(ref))
    # the same comparison fails for the swapped assembly (U1 <-> U2)
    th2 = th.copy()
    Q = model.unpack(spec, th2)
    Q["U1"][:], Q["U2"][:] = P["U2"].copy(), P["U1"].copy()
    lp2 = model.log_psi(spec, th2, sig)
    assert np.max(np.abs(2 * lp2.real - ref)) > 1e-3
    # ... and for sigma' = [sigma_v; sigma_h] (spin columns swapped)
    th3 = th.copy()
    R = model.unpack(spec, th3)
    for name, c0 in (("Wu", H), ("Wr", H), ("Win", 0)):
        a, b = R[name][:, c0:c0 + 2].copy(), R[name][:, c0 + 2:c0 + 4].copy()
        R[name][:, c0:c0 + 2], R[name][:, c0 + 2:c0 + 4] = b, a
    lp3 = model.log_psi(spec, th3, sig)
    assert np.max(np.abs(2 * lp3.real - ref)) > 1e-3


def test_momentum_by_hand():
    # App. B: m_{t+1} = mu m_t + (1 - mu) dtheta_t, theta_{t+1} = theta_t -
    # m_{t+1}; two steps at mu = 0.75 with dyadic values worked out by hand
    th0 = np.array([1.0, -2.0])
    m0 = np.zeros(2)
    th1, m1 = minsr.momentum(th0, m0, np.array([0.5, 0.25]), 0.75)
    assert np.array_equal(m1, [0.125, 0.0625])
    assert np.array_equal(th1, [0.875, -2.0625])
    th2, m2 = minsr.momentum(th1, m1, np.array([-1.0, 2.0]), 0.75)
    assert np.array_equal(m2, [-0.15625, 0.546875])
    assert np.array_equal(th2, [1.03125, -2.609375])


def test_momentum_geometric_series():
    # a constant direction d from m_0 = 0 gives m_t = (1 - mu^t) d (the
    # geometric series of App. B's recursion); mu = 0.7 over 12 steps
    d = np.array([0.3, -1.7, 2.5])
    th, m = np.zeros(3), np.zeros(3)
    mu = 0.7
    for t in range(1, 13):
        th, m = minsr.momentum(th, m, d, mu)
        assert np.allclose(m, (1.0 - mu ** t) * d, rtol=1e-14, atol=0)
    # theta_t = -sum_s m_s = -(t - mu (1 - mu^t) / (1 - mu)) d
    assert np.allclose(th, -(12 - mu * (1 - mu ** 12) / (1 - mu)) * d, rtol=1e-13, atol=0)


# ------------------------------------------------ adaptive regularisation

from oracle import adaptive  # noqa: E402


@pytest.mark.parametrize("cplx", [False, True])
def test_tnorm_is_parameter_space_norm(cplx):
    # ||T||_F = ||S||_F (T and S = O' O'^T share their non-zero spectrum) and
    # equals the 2-norm of T's eigenvalues
    _, _, D, eps = _config1_inputs(cplx)
    r = minsr.update(D, eps, 0.01, 1e-3)
    tn = adaptive.tnorm(r["T"])
    S = r["Op"] @ r["Op"].T
    assert abs(tn - np.linalg.norm(S, "fro")) < 1e-12 * tn
    assert abs(tn - np.sqrt(np.sum(np.linalg.eigvalsh(r["T"]) ** 2))) < 1e-12 * tn


def test_pow23_by_hand():
    # ||diag(4, 4, 4, 4)||_F = 8, 8^{2/3} = 4: lambda = 3e-4 * 4 (Sec. 3.3)
    T = np.diag([4.0, 4.0, 4.0, 4.0])
    assert adaptive.tnorm(T) == 8.0
    assert abs(adaptive.lambda_pow23(T, 3e-4) - 1.2e-3) < 1e-18


@pytest.mark.parametrize("pinv", [False, True])
def test_trust_region_saturates_constraint(pinv):
    # App. F: the step eta_* O' x has dtheta^T S dtheta = eta^2 with the
    # parameter-space metric S = O' O'^T formed densely (N_p = 962), and
    # ||tau|| is the paper's ||(I - lambda (T + lambda I)^{-1}) e'|| with an
    # explicit inverse (Cholesky) or ||T T^+ e'|| (pseudo-inverse)
    _, _, D, eps = _config1_inputs(False)
    eta = 0.07
    lam, cut = (0.0, 1e-8) if pinv else (1e-3, 0.0)
    r = minsr.update(D, eps, 1.0, lam, pinv_cutoff=cut)
    T, ep, x, Op = r["T"], r["ep"], r["x"], r["Op"]
    tau = adaptive.tau_vector(T, ep, x, lam, pinv)
    n = T.shape[0]
    if pinv:
        ref = T @ (np.linalg.pinv(T, rcond=1e-8, hermitian=True) @ ep)
    else:
        ref = (np.eye(n) - lam * np.linalg.inv(T + lam * np.eye(n))) @ ep
    assert np.max(np.abs(tau - ref)) < 1e-9 * np.max(np.abs(ref))
    eta_s = eta / np.linalg.norm(tau)
    dth = eta_s * (Op @ x)
    S = Op @ Op.T
    assert abs(dth @ S @ dth - eta ** 2) < 1e-9 * eta ** 2


def test_lm_denominator_is_quadratic_model():
    # App. G: g^T dtheta - dtheta^T S dtheta / 2 with g = O' e' and
    # S = O' O'^T formed densely, for a plain and a trust-region rate
    _, _, D, eps = _config1_inputs(True)
    lam = 2e-3
    r = minsr.update(D, eps, 1.0, lam)
    T, ep, x, Op = r["T"], r["ep"], r["x"], r["Op"]
    tau = adaptive.tau_vector(T, ep, x, lam, False)
    g = Op @ ep
    S = Op @ Op.T
    for eta_used in (0.01, 0.05 / np.linalg.norm(tau)):
        dth = eta_used * (Op @ x)
        pred = g @ dth - 0.5 * dth @ S @ dth
        assert abs(adaptive.predicted_decrease(eta_used, ep, tau) - pred) < 1e-10 * abs(pred)


def test_lm_ratio_tends_to_one_with_exact_energies():
    # On a wave function whose distribution is uniform (zero output weights
    # and biases) the full enumeration of configurations is an exact
    # "sample set": then g is the exact energy gradient, and with exact
    # energies E(theta) and E(theta - dtheta) from the dense Hamiltonian the
    # ratio is 1 + O(eta) (App. G's quadratic model to first order).
    N = 6
    spec = model.Spec(Lx=N, H=4, complex_head=True)
    th = scaled_theta(spec, 71, 1.0)
    P = model.unpack(spec, th)
    P["U"][:] = 0.0
    P["c"][:] = 0.0
    s = refs.all_configs(N)
    ham = ham_mod.Ham("tfim", J=1.0, h=0.7)
    Hd = refs.dense_tfim(N, 1.0, 0.7, False)

    def energy(t):
        psi = np.exp(model.log_psi(spec, t, s))
        return float((np.conj(psi) @ (Hd @ psi)).real / (np.conj(psi) @ psi).real)

    lp = model.log_psi(spec, th, s)
    assert np.allclose(np.exp(2 * lp.real), 1.0 / 2 ** N, rtol=1e-13)
    eps = ham_mod.local_energy(spec, th, ham, s, lp)
    D = jacobian.log_derivatives(spec, th, s)
    lam = 1e-3
    r = minsr.update(D, eps, 1.0, lam)
    tau = adaptive.tau_vector(r["T"], r["ep"], r["x"], lam, False)
    E0 = energy(th)
    assert abs(E0 - r["E"].real) < 1e-12
    dev = []
    for eta in (1e-2, 1e-3):
        rho = adaptive.lm_ratio(E0, energy(th - eta * r["dtheta"]), eta, r["ep"], tau)
        dev.append(abs(rho - 1.0))
    assert dev[1] < 0.02
    assert dev[1] < 0.2 * dev[0]      # first order in eta


def test_lm_lambda_rule_by_hand():
    # App. G with omega = 3/2: strict inequalities at 1/4 and 3/4
    assert adaptive.lm_next(1e-2, 0.1, 1.5) == 1.5e-2
    assert adaptive.lm_next(1e-2, -3.0, 1.5) == 1.5e-2
    assert adaptive.lm_next(1e-2, 0.9, 1.5) == 1e-2 / 1.5
    assert adaptive.lm_next(1e-2, 0.5, 1.5) == 1e-2
    assert adaptive.lm_next(1e-2, 0.25, 1.5) == 1e-2
    assert adaptive.lm_next(1e-2, 0.75, 1.5) == 1e-2
    assert adaptive.lm_next(1e-2, float("nan"), 1.5) == 1.5e-2


def test_adaptive_step_reduces_to_plain_step():
    # constant lambda without the trust region is Alg. 1's step
    spec = model.Spec(Lx=8, H=8)
    th = scaled_theta(spec, 72, 1.0)
    ham = ham_mod.Ham("tfim", J=1.0, h=1.0, pbc=True)
    a = adaptive.step(spec, th, np.zeros_like(th), ham, 40, 0.02, 1e-3, 0.3, 5, 2)
    b = minsr.step(spec, th, np.zeros_like(th), ham, 40, 0.02, 1e-3, 0.3, 5, 2)
    assert np.array_equal(a["dtheta"], b["dtheta"])
    assert np.array_equal(a["theta"], b["theta"])
    assert a["eta_used"] == 0.02 and a["lam_used"] == 1e-3


# ------------------------------------------------ conditioning (App. E)

from oracle import conditioning  # noqa: E402


def test_condition_by_hand():
    # diag(4, 1, 0), lambda = 1: kappa_2 = (4 + 1) / (0 + 1) = 5 and
    # d = -log10(5 * 1e-7) = 7 - log10(5)
    T = np.diag([4.0, 1.0, 0.0])
    wmin, wmax, k, d = conditioning.condition(T, 1.0, 1e-7)
    assert (wmin, wmax, k) == (0.0, 4.0, 5.0)
    assert abs(d - (7.0 - math.log10(5.0))) < 1e-14
    # no shift on a singular matrix: infinite condition, no reliable digit
    assert conditioning.kappa2(np.array([0.0, 2.0]), 0.0) == math.inf
    assert conditioning.digits(math.inf, 1e-16) == -math.inf


@pytest.mark.parametrize("cplx", [False, True])
def test_condition_matches_svd_condition_number(cplx):
    # kappa_2 of T + lambda I from the spectrum equals the 2-norm condition
    # number from the singular values (numpy's cond), and the spectrum has
    # the trace and Frobenius norm of T
    _, _, D, eps = _config1_inputs(cplx)
    r = minsr.update(D, eps, 0.01, 1e-3)
    T = r["T"]
    for lam in (1e-3, 1e-1):
        _, _, k, _ = conditioning.condition(T, lam, 2.0 ** -52)
        ref = np.linalg.cond(T + lam * np.eye(T.shape[0]), 2)
        assert abs(k - ref) < 1e-8 * ref
    w = conditioning.spectrum(T)
    assert abs(w.sum() - np.trace(T)) < 1e-10 * np.trace(T)
    assert abs(np.sqrt((w * w).sum()) - np.linalg.norm(T)) < 1e-10 * np.linalg.norm(T)
    assert np.all(np.diff(w) >= 0)


# ------------------------------------------------ subsampled QGT (Prop. 3)

from oracle import qgt  # noqa: E402


def test_subsampled_S_is_real_part_of_empirical_qgt():
    # Eq. SR: O' O'^T of the real form equals Re[(1/Ns) sum (O - Obar)(O - Obar)^dagger]
    _, _, D, _ = _config1_inputs(True)
    S = qgt.subsampled_S(D)
    Xc = D - D.mean(axis=0)
    ref = np.real(Xc.T @ np.conj(Xc)) / D.shape[0]
    assert np.max(np.abs(S - ref)) < 1e-12 * np.max(np.abs(ref))


def test_qgt_estimator_mean_square_error_and_bound():
    # i.i.d. draws from the exact Born distribution (N = 6 chain, cRNN):
    # E ||Q - Q~||_F^2 = N_p^2 V_avg / N_s exactly (the identity behind
    # Prop. 3), and the probability of exceeding the bound at epsilon stays
    # below epsilon
    spec = model.Spec(Lx=6, H=3, complex_head=True)
    th = scaled_theta(spec, 73, 1.5)
    pop = qgt.population(spec, th)
    P = pop["P"]
    assert abs(P.sum() - 1.0) < 1e-12
    Np = pop["X"].shape[1]
    rng = np.random.default_rng(5)
    Ns, sets = 8, 3000
    sq = np.empty(sets)
    for t in range(sets):
        idx = rng.choice(len(P), size=Ns, p=P)
        sq[t] = np.linalg.norm(pop["Q"] - qgt.estimate(pop["X"][idx])) ** 2
    expect = Np ** 2 * pop["V_avg"] / Ns
    se = sq.std() / math.sqrt(sets)
    assert abs(sq.mean() - expect) < 4 * se, (sq.mean(), expect, se)
    for epsilon in (0.1, 0.3):
        b = qgt.bound(Np, Ns, pop["V_avg"], epsilon)
        assert np.mean(np.sqrt(sq) > b) <= epsilon
