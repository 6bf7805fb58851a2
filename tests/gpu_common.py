"""Helpers shared by the GPU parity tests: build a GPU model and an oracle
spec of the same architecture, move parameters between them."""
import numpy as np
import pytest
import torch

from oracle import model as omodel

gpu = pytest.mark.gpu


def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")


def make_pair(Lx, Ly=1, dim=1, H=16, cplx=False, marshall=False, zero_mag=False, dtype="f64",
              seed=2001, max_Ns=256):
    import paper_2608_18065_amd as pm
    spec = omodel.Spec(Lx=Lx, Ly=Ly, dim=dim, H=H, complex_head=cplx, marshall=marshall,
                       zero_mag=zero_mag)
    m = pm.Model(Lx, Ly, dim, H, cplx, marshall, zero_mag, dtype=dtype, seed=seed, max_Ns=max_Ns)
    assert m.Np == omodel.num_params(spec)
    return spec, m


def scaled_theta(spec, seed, scale):
    """Glorot init with weights scaled up (conditionals far from uniform)
    and non-zero biases."""
    th = omodel.glorot_init(spec, seed) * scale
    rng = np.random.default_rng(seed)
    off = 0
    for name, shape in omodel.layout(spec):
        n = int(np.prod(shape))
        if len(shape) == 1:
            th[off:off + n] = rng.uniform(-0.5, 0.5, n)
        off += n
    return th


def to_dev(a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def rel_err(a, b):
    """Largest entrywise difference relative to the largest entry of the
    reference: max|a - b| / max|b| (the floor only avoids 0 / 0)."""
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.max(np.abs(a - b)) / max(1e-300, float(np.max(np.abs(b)))))


def _draw_margins(spec, th, sigma, u):
    """|u - p_i(0)| at every site of the given draws, with p_i(0) the
    oracle's FP64 conditional along the drawn configuration."""
    from oracle import model as omodel
    run = omodel.run(spec, th, sigma=sigma)
    P = omodel.unpack(spec, th)
    Ns, N = sigma.shape
    nup = np.zeros(Ns, dtype=np.int64)
    ndn = np.zeros(Ns, dtype=np.int64)
    out = np.empty((Ns, N))
    for k in range(N):
        _, p, _ = omodel.conditional(spec, P, run["hs"][:, k], nup, ndn)
        out[:, k] = np.abs(u[:, k] - p[:, 0])
        nup += sigma[:, k] == 0
        ndn += sigma[:, k] == 1
    return out


# an FP32 conditional is within a few FP32 ulps of the FP64 one; a draw
# whose uniform lies closer than this to the conditional is a tie
FP32_TIE = 1e-6


def low_precision_step(spec, m, gham, ham, Ns, eta, lam, key, counter, form, ckpt_every=1,
                       pinv_cutoff=0.0):
    """One step of a low-precision form against the FP64 oracle.  The FP32
    sampler may only differ from the FP64 draws where the uniform ties with
    the conditional to FP32 resolution: then the first differing site of
    each differing sample must be such a tie, and the oracle's downstream
    stages are re-run on the GPU's samples.  Anything else fails.
    gham: the library's Hamiltonian; ham: the oracle's."""
    mom = torch.zeros(m.Np, dtype=torch.float64, device="cuda")
    th = m.get_params().cpu().numpy()
    o = m.step(gham, Ns, eta, lam, 0.0, mom, key, counter, form=form, ckpt_every=ckpt_every,
               pinv_cutoff=pinv_cutoff)
    torch.cuda.synchronize()
    return o, low_precision_ref(spec, th, ham, Ns, eta, lam, key, counter, o, pinv_cutoff)


def low_precision_ref(spec, th, ham, Ns, eta, lam, key, counter, o, pinv_cutoff=0.0):
    """The oracle's step (momentum 0) from parameters th for the outputs o
    of a low-precision step already taken on the GPU, with the tie rule of
    low_precision_step for samples that differ."""
    import paper_2608_18065_amd as pm
    from oracle import hamiltonian as oham
    from oracle import jacobian as ojac
    from oracle import minsr as ominsr
    from oracle import philox
    assert int(o["status"].item()) & pm.ST_ERRORS == 0
    ref = ominsr.step(spec, th, np.zeros_like(th), ham, Ns, eta, lam, 0.0, key, counter,
                      pinv_cutoff=pinv_cutoff)
    u = philox.uniforms(key, counter, Ns, spec.N)
    sig = o["sigma"].cpu().numpy()
    diff = sig != ref["sigma"].astype(np.uint8)
    margin = _draw_margins(spec, th, ref["sigma"], u)
    if not diff.any():
        return ref
    rows = np.nonzero(diff.any(axis=1))[0]
    assert len(rows) <= max(2, Ns // 200), "%d samples differ" % len(rows)
    for r in rows:
        k = int(np.argmax(diff[r]))
        assert margin[r, k] < FP32_TIE, (r, k, margin[r, k])
    # the oracle's stages on the GPU's samples (same arithmetic as its step)
    lp = omodel.log_psi(spec, th, sig.astype(np.int64))
    eps = oham.local_energy(spec, th, ham, sig.astype(np.int64), lp)
    D = ojac.log_derivatives(spec, th, sig.astype(np.int64))
    ref = ominsr.update(D, eps, eta, lam, pinv_cutoff)
    ref.update(sigma=sig, eps=eps)
    return ref
