"""Parity at the full model sizes of the benchmark systems (full N, d_h and
architecture, so every kernel takes the path it takes there; fewer samples so
the FP64 oracle stays tractable): the cluster chain (N = 100, d_h = 128 cRNN,
checkpoints every 10 sites), the 10 x 10 Heisenberg lattice (2D pRNN,
Marshall sign, S^z = 0 mask, pseudo-inverse), one 12 x 12 J1-J2 instance of
the batched workload, batch replays against the oracle (FP64 instances, and
BF16 instances of the batched workload's architecture whose Grams run in one
grouped launch), and the pseudo-inverse at n = 4096."""
import numpy as np
import pytest
import torch

from oracle import hamiltonian as oham
from oracle import minsr as ominsr
from oracle import model as omodel
from tests import inputs
from tests.gpu_common import (gpu, low_precision_ref, low_precision_step, make_pair, need_gpu,
                              rel_err, to_dev)

pytestmark = gpu


@pytest.fixture(autouse=True)
def _gpu():
    need_gpu()


def _gham(h):
    import paper_2608_18065_amd as pm
    return pm.hamiltonian(h.kind, J=h.J, h=h.h, J2=h.J2, pbc=h.pbc)


def _frob(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _compare_low_precision(o, ref, it, form, tol_dtheta=2e-2):
    import paper_2608_18065_amd as pm
    E = o["energy"].cpu().numpy()
    assert abs(E[0] - ref["E"].real) < 1e-4 * abs(ref["E"].real)
    ep = it["eps_prime"].cpu().numpy()
    assert np.max(np.abs(ep - ref["ep"])) < 1e-4 * np.max(np.abs(ref["ep"]))
    T = it["T"].double().cpu().numpy()
    errT = _frob(T, ref["T"])
    assert errT < 2e-2, errT
    R = it["Oprime"].double().cpu().numpy()
    if form == pm.FORM_BF16_FP64:
        R = R + it["Oprime_lo"].double().cpu().numpy()
    errR = rel_err(R, ref["Op"].T)
    assert errR < 1e-4, errR
    errd = None
    if tol_dtheta is not None:
        d = o["dtheta"].cpu().numpy()
        errd = _frob(d, ref["dtheta"])
        assert errd < tol_dtheta, errd
    return errT, errR, errd


def test_cluster100_full_size_bf16_step():
    # N = 100 periodic cluster chain, 1D cRNN d_h = 128 (50948 parameters),
    # FP32 recurrence, checkpoints every 10 sites, BF16 + FP64 form
    import paper_2608_18065_amd as pm
    from workloads import WORKLOADS
    wl = WORKLOADS["cluster100"]
    Ns = 256
    print("cluster100 full size, Ns=%d" % Ns, flush=True)
    spec, m = make_pair(Lx=wl.Lx, H=wl.H, cplx=True, dtype="f32", seed=wl.seed, max_Ns=Ns)
    assert m.Np == 50948
    ham = oham.Ham("cluster")
    o, ref = low_precision_step(spec, m, _gham(ham), ham, Ns, wl.eta, wl.lam, wl.key, 0,
                                pm.FORM_BF16_FP64, ckpt_every=wl.ckpt_every)
    it = m.intermediates(pm.FORM_BF16_FP64)
    print("errors T %.2e  O' %.2e  dtheta %.2e" % _compare_low_precision(
        o, ref, it, pm.FORM_BF16_FP64), flush=True)


def test_heis10x10_full_size_pinv_step():
    # 10 x 10 open Heisenberg lattice, 2D pRNN d_h = 128 (84226 parameters)
    # with Marshall sign and S^z = 0 masking, BF16 Gram, FP64 pseudo-inverse
    # at lambda = 0 with the relative cutoff 1e-8.  The BF16 Gram resolves
    # the eigenvalues near the cutoff only to its own accuracy, so dtheta is
    # checked against the pseudo-inverse step evaluated in FP64 on the GPU's
    # own T, eps' and O' (the solve and update at this size), the rest
    # against the oracle's step
    import paper_2608_18065_amd as pm
    from workloads import WORKLOADS
    wl = WORKLOADS["heis10x10"]
    Ns = 128
    print("heis10x10 full size, Ns=%d" % Ns, flush=True)
    spec, m = make_pair(Lx=10, Ly=10, dim=2, H=128, marshall=True, zero_mag=True, dtype="f32",
                        seed=wl.seed, max_Ns=Ns)
    assert m.Np == 84226
    ham = oham.Ham("j1j2", J=1.0, J2=0.0)
    o, ref = low_precision_step(spec, m, _gham(ham), ham, Ns, wl.eta, 0.0, wl.key, 0,
                                pm.FORM_BF16_FP64, pinv_cutoff=wl.pinv_cutoff)
    it = m.intermediates(pm.FORM_BF16_FP64)
    errT, errR, _ = _compare_low_precision(o, ref, it, pm.FORM_BF16_FP64, tol_dtheta=None)
    T = it["T"].cpu().numpy()
    ep = it["eps_prime"].cpu().numpy()
    R = it["Oprime"].double().cpu().numpy() + it["Oprime_lo"].double().cpu().numpy()
    w = np.linalg.eigvalsh(T)
    thr = wl.pinv_cutoff * w.max()
    assert np.all(np.abs(w - thr) > 1e-6 * thr), "ambiguous cutoff for this seed"
    x = ominsr.solve(T, ep, 0.0, wl.pinv_cutoff)
    d_ref = wl.eta * (R.T @ x)
    kept = w[w > thr]
    tol = max(1e-10, 4.0 * Ns * np.finfo(float).eps * w.max() / kept.min())
    d = o["dtheta"].cpu().numpy()
    errd = _frob(d, d_ref)
    print("errors T %.2e  O' %.2e  dtheta (own T) %.2e (tol %.1e)" % (errT, errR, errd, tol))
    assert errd < tol


def test_j1j2_12x12_full_size_bf16_step():
    # the largest instance of the batched J1-J2 workload: 12 x 12 open
    # lattice, J2 = 0.5, 2D cRNN d_h = 128 with Marshall sign, lambda = 0.1
    import paper_2608_18065_amd as pm
    from workloads import j1j2_batch
    wl = [w for w in j1j2_batch() if w.Lx == 12][0]
    Ns = 64
    print("j1j2 12x12 full size, Ns=%d" % Ns, flush=True)
    spec, m = make_pair(Lx=12, Ly=12, dim=2, H=128, cplx=True, marshall=True, dtype="f32",
                        seed=wl.seed, max_Ns=Ns)
    ham = oham.Ham("j1j2", J=1.0, J2=0.5)
    o, ref = low_precision_step(spec, m, _gham(ham), ham, Ns, wl.eta, wl.lam, wl.key, 0,
                                pm.FORM_BF16_FP64)
    it = m.intermediates(pm.FORM_BF16_FP64)
    print("errors T %.2e  O' %.2e  dtheta %.2e" % _compare_low_precision(
        o, ref, it, pm.FORM_BF16_FP64), flush=True)


def test_batch_replay_matches_oracle():
    # one replay of a captured batch of two FP64 instances (a periodic TFIM
    # chain and a complex J1-J2 lattice) against the oracle's steps
    import paper_2608_18065_amd as pm
    cases = [(dict(Lx=12, H=16), oham.Ham("tfim", J=1.0, h=0.9, pbc=True), 80, 501),
             (dict(Lx=3, Ly=4, dim=2, H=16, cplx=True, marshall=True),
              oham.Ham("j1j2", J=1.0, J2=0.5), 60, 502)]
    insts, pairs = [], []
    for arch, ham, Ns, key in cases:
        spec, m = make_pair(**arch, max_Ns=Ns, seed=key)
        pairs.append((spec, m, ham, Ns, key))
        insts.append(dict(model=m, ham=_gham(ham), Ns=Ns, eta=0.05, lam=1e-2, mu=0.3, key=key,
                          form=pm.FORM_FP64_REF))
    th0 = [m.get_params().cpu().numpy() for _, m, _, _, _ in pairs]
    b = pm.Batch(insts)
    b.step()
    torch.cuda.synchronize()
    for k, (spec, m, ham, Ns, key) in enumerate(pairs):
        ref = ominsr.step(spec, th0[k], np.zeros_like(th0[k]), ham, Ns, 0.05, 1e-2, 0.3, key, 0)
        ob = b.outputs[k]
        assert int(ob["status"].item()) == 0
        assert np.array_equal(ob["sigma"].cpu().numpy(), ref["sigma"].astype(np.uint8))
        assert rel_err(ob["dtheta"].cpu().numpy(), ref["dtheta"]) < 1e-10
        assert rel_err(b.momentum[k].cpu().numpy(), ref["m"]) < 1e-10
    b.close()


def test_batch_grouped_gram_matches_oracle():
    # one replay of a batch of three instances of the batched J1-J2
    # workload's architecture (2D cRNN d_h = 128, Marshall sign, J2 = 0.5) on
    # 6 x 6, 7 x 7 and 5 x 5 lattices with uneven N_s, all in the BF16 split
    # form: their Grams run as one grouped launch.  Every instance's T,
    # eps', O' and dtheta against the oracle's step
    import paper_2608_18065_amd as pm
    ham = oham.Ham("j1j2", J=1.0, J2=0.5)
    cases = [(6, 128, 701), (7, 96, 702), (5, 150, 703)]
    insts, pairs = [], []
    for L, Ns, key in cases:
        print("grouped batch instance %dx%d Ns=%d" % (L, L, Ns), flush=True)
        spec, m = make_pair(Lx=L, Ly=L, dim=2, H=128, cplx=True, marshall=True, dtype="f32",
                            seed=key, max_Ns=Ns)
        pairs.append((spec, m, Ns, key))
        insts.append(dict(model=m, ham=_gham(ham), Ns=Ns, eta=0.1, lam=0.1, mu=0.0, key=key,
                          form=pm.FORM_BF16_FP64))
    th0 = [m.get_params().cpu().numpy() for _, m, _, _ in pairs]
    b = pm.Batch(insts)
    b.step()
    torch.cuda.synchronize()
    for k, (spec, m, Ns, key) in enumerate(pairs):
        ref = low_precision_ref(spec, th0[k], ham, Ns, 0.1, 0.1, key, 0, b.outputs[k])
        it = m.intermediates(pm.FORM_BF16_FP64)
        print("instance %d: errors T %.2e  O' %.2e  dtheta %.2e" % ((k,) + _compare_low_precision(
            b.outputs[k], ref, it, pm.FORM_BF16_FP64)), flush=True)
    b.close()


def test_pinv_n4096_designed_spectrum():
    # the pseudo-inverse at the size of the 10 x 10 workload's sample space
    import paper_2608_18065_amd as pm
    n, cutoff = 4096, 1e-8
    m = pm.Model(16, hidden=8, dtype="f64", seed=1, max_Ns=n, pinv=True)
    rng = np.random.default_rng(4096)
    w = inputs.spectrum_loguniform(n, 1e6, rng, zeros=n // 8)
    T, _ = inputs.psd_matrix(w, seed=4097)
    b = inputs.rhs(n, seed=4098)
    wo = np.linalg.eigvalsh(T)
    thr = cutoff * wo.max()
    assert np.all(np.abs(wo - thr) > 1e-6 * thr)
    x, st = m.solve(to_dev(T), to_dev(b), lam=0.0, pinv_cutoff=cutoff)
    torch.cuda.synchronize()
    assert int(st.item()) == 0
    ref = ominsr.solve(T, b, 0.0, cutoff)
    kept = wo[wo > thr]
    tol = max(1e-10, 4.0 * n * np.finfo(float).eps * wo.max() / kept.min())
    err = _frob(x.cpu().numpy(), ref)
    print("pinv n=4096: rel err %.2e (tol %.1e)" % (err, tol))
    assert err < tol
    m.close()
